"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (fixed by the accuracy target of the method): complex64 runs
match within 1e-5 absolute on expectations and states and 1e-4 absolute on
gradients; complex128 runs within 1e-10. Inputs are the seeded workloads of
``workloads`` and seeded random circuits over every gate kind.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from workloads import circuits as C
from workloads import data as Dt
from _patterns import cnot_pattern
from _channels import stable_uniforms, channel_gates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2509_25075_amd import _native as N
    from paper_2509_25075_amd import sim

TOL = {"c64": dict(z=1e-5, state=1e-5, grad=1e-4),
       "c128": dict(z=1e-10, state=1e-10, grad=1e-10)}
PATHS = {"fused": 1, "plain": 2, "hbm": 3, "auto": 0, "mfma": 4}


def _dev(a, dt):
    return None if a is None else torch.as_tensor(np.asarray(a)).to("cuda", dt).contiguous()


def _announce(msg):
    print(msg, flush=True)


def _run_expz_case(c, dtype, path, B, seed, per_sample=False, amplitude=True,
                   dstate_mode=False):
    """Forward (state + <Z>) and adjoint on the GPU vs the oracle."""
    _announce(f"case n={c.n_qubits} G={c.n_gates} B={B} {dtype} {path} "
              f"ps={per_sample} dstate={dstate_mode}")
    rng = np.random.default_rng(seed)
    n = c.n_qubits
    rd = np.float32 if dtype == "c64" else np.float64
    P = c.n_params
    params = rng.uniform(-np.pi, np.pi, (B, P) if per_sample else P).astype(rd)
    feats = rng.uniform(-1, 1, (B, c.n_features)).astype(rd) if c.n_features else None
    flags = PATHS[path] | (N.QS_FLAG_PER_SAMPLE_PARAMS if per_sample else 0)
    s = sim.Simulator(c, dtype, flags)
    if amplitude:
        D = max(1, (1 << n) - (1 << n) // 3)  # zero-padded tail
        x = rng.standard_normal((B, D)).astype(rd)
        psi0 = O.encode_amplitude(x, n)
        st = s.encode_amplitude(_dev(x, s.rdtype))
    else:
        psi0 = O.encode_zero(B, n)
        st = s.zero_state(B)
    st0 = st.clone()
    pt, ft = _dev(params, s.rdtype), _dev(feats, s.rdtype)
    z = s.forward(pt, ft, st)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    psiG = O.run_circuit(c, params, feats, psi0)
    np.testing.assert_allclose(st0.cpu().numpy(), psi0, atol=tol["state"])
    np.testing.assert_allclose(st.cpu().numpy(), psiG, atol=tol["state"])
    np.testing.assert_allclose(z.cpu().numpy(), O.expz(psiG), atol=tol["z"])
    if dstate_mode:
        lam = (rng.standard_normal((B, 1 << n)) + 1j * rng.standard_normal((B, 1 << n))) * 0.3
        gp, gf = s.adjoint(pt, ft, st, dstate=_dev(lam, s.cdtype))
        gth, _ = O.adjoint_vjp(c, params, feats, psi0, lam_final=lam)
    else:
        dz = rng.uniform(-1, 1, (B, n))
        gp, gf = s.adjoint(pt, ft, st, dexpz=_dev(dz, torch.float64))
        gth, _ = O.adjoint_vjp(c, params, feats, psi0, dexpz=dz)
    torch.cuda.synchronize()
    rp, rf = O.theta_to_param_grads(c, params, feats, gth)
    np.testing.assert_allclose(gp.cpu().numpy(), rp, atol=tol["grad"])
    if feats is not None:
        np.testing.assert_allclose(gf.cpu().numpy(), rf, atol=tol["grad"])


# ------------------------------------------------------------ random circuits
@pytest.mark.parametrize("path", ["fused", "plain"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14])
def test_random_circuit_c64(n, path):
    rng = np.random.default_rng(100 + n)
    c = C.random_circuit(n, 90, rng, n_params=7, n_features=3)
    B = 37 if n <= 10 else 5
    _run_expz_case(c, "c64", path, B, seed=n)


@pytest.mark.parametrize("path", ["fused", "plain"])
@pytest.mark.parametrize("n", [1, 3, 4, 6, 9, 12, 13])
def test_random_circuit_c128(n, path):
    rng = np.random.default_rng(200 + n)
    c = C.random_circuit(n, 70, rng, n_params=5, n_features=2)
    _run_expz_case(c, "c128", path, 11 if n <= 9 else 3, seed=n)


# Circuits whose every block is RY then RZ run the adjoint's gate-at-a-time
# pass (register tiles 2^4 and 2^5 in complex64, 2^4 in complex128); the
# builders give such circuits (re-uploading adds features to the RY angles).
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("kind,n", [("ring", 1), ("ring", 3), ("ring", 5), ("ring", 9),
                                    ("ring", 12), ("ring", 14), ("chain", 7), ("chain", 11),
                                    ("reupload", 6), ("reupload", 10), ("ring", 16)])
def test_ry_rz_circuits(kind, n, dtype):
    if kind == "ring":
        c = C.hea_ry_rz_ring(n, 3)
    elif kind == "chain":
        c = C.ry_rz_chain(n, 3)
    else:
        c = C.reupload_ry_rz_chain(n, 3, 3)
    B = 21 if n <= 10 else 3
    _run_expz_case(c, dtype, "auto", B, seed=1800 + n)
    if n <= 13:
        _run_expz_case(c, dtype, "auto", B, seed=1900 + n, per_sample=True)


# Feature gradients of complex64 per-sample blocks with at most four
# features accumulate per lane in registers; with more they take the
# per-gate LDS sums. Both, on random circuits (general and two-gate blocks)
# and on re-uploading layers (the RY-then-RZ pass).
@pytest.mark.parametrize("nf", [1, 4, 5, 7])
@pytest.mark.parametrize("n", [4, 9, 12])
def test_feature_counts(n, nf):
    rng = np.random.default_rng(2300 + 10 * n + nf)
    B = 17 if n <= 9 else 3
    _announce(f"feature counts n={n} features={nf}")
    _run_expz_case(C.random_circuit(n, 70, rng, n_params=6, n_features=nf), "c64", "fused", B,
                   seed=n + nf)
    _run_expz_case(C.reupload_ry_rz_chain(n, 2, nf), "c64", "auto", B, seed=n + 3 * nf)


@pytest.mark.parametrize("path", ["fused", "plain"])
@pytest.mark.parametrize("n", [2, 6, 10, 13])
def test_per_sample_params(n, path):
    rng = np.random.default_rng(300 + n)
    c = C.random_circuit(n, 60, rng, n_params=6, n_features=2)
    _run_expz_case(c, "c64", path, 19 if n <= 10 else 3, seed=n, per_sample=True)


@pytest.mark.parametrize("path", ["fused", "plain"])
@pytest.mark.parametrize("n", [3, 8, 11])
def test_state_cotangent(n, path):
    rng = np.random.default_rng(400 + n)
    c = C.random_circuit(n, 60, rng, n_params=6, n_features=2)
    _run_expz_case(c, "c64", path, 13 if n <= 8 else 3, seed=n, dstate_mode=True,
                   amplitude=False)


def _reversed(c):
    """U^dagger written out: gates reversed, rotation scales negated."""
    g = c.gates[::-1].copy()
    rot = np.isin(g["op"], (C.OP["RX"], C.OP["RY"], C.OP["RZ"]))
    g["scale"][rot] = -g["scale"][rot]
    return C.Circuit(c.n_qubits, g, c.n_params, c.n_features)


@pytest.mark.parametrize("n,path", [(7, "fused"), (7, "plain"), (16, "auto")])
def test_inverse_flag(n, path):
    """QS_FLAG_INVERSE runs U^dagger: it undoes a forward sweep, and its forward
    and adjoint match the oracle on the reversed, negated gate list."""
    rng = np.random.default_rng(800 + n)
    c = C.random_circuit(n, 60, rng, n_params=5, n_features=2)
    B = 9 if n <= 10 else 2
    _announce(f"inverse flag n={n} {path} B={B}")
    params = rng.uniform(-np.pi, np.pi, c.n_params).astype(np.float32)
    feats = rng.uniform(-1, 1, (B, 2)).astype(np.float32)
    x = rng.standard_normal((B, 1 << n)).astype(np.float32)
    s = sim.Simulator(c, "c64", PATHS[path])
    si = sim.Simulator(c, "c64", PATHS[path] | N.QS_FLAG_INVERSE)
    pt, ft = _dev(params, torch.float32), _dev(feats, torch.float32)
    st = s.encode_amplitude(_dev(x, torch.float32))
    st0 = st.clone()
    s.forward(pt, ft, st)
    si.forward(pt, ft, st)
    torch.cuda.synchronize()
    np.testing.assert_allclose(st.cpu().numpy(), st0.cpu().numpy(), atol=1e-5)
    rev = _reversed(c)
    psi0 = O.encode_amplitude(x, n)
    psiG = O.run_circuit(rev, params, feats, psi0)
    z = si.forward(pt, ft, st)          # st holds psi0 again
    dz = rng.uniform(-1, 1, (B, n))
    gp, gf = si.adjoint(pt, ft, st, dexpz=_dev(dz, torch.float64))
    torch.cuda.synchronize()
    np.testing.assert_allclose(st.cpu().numpy(), psiG, atol=1e-5)
    np.testing.assert_allclose(z.cpu().numpy(), O.expz(psiG), atol=1e-5)
    gth, _ = O.adjoint_vjp(rev, params, feats, psi0, dexpz=dz)
    rp, rf = O.theta_to_param_grads(rev, params, feats, gth)
    np.testing.assert_allclose(gp.cpu().numpy(), rp, atol=1e-4)
    np.testing.assert_allclose(gf.cpu().numpy(), rf, atol=1e-4)


def test_empty_circuit_and_single_gate():
    for rows in ([], [(C.OP["RY"], 0, -1, 0, -1, -1, 1.0, 0)]):
        c = C.Circuit(3, np.array(rows, dtype=C.GATE_DTYPE), 1)
        for path in ("fused", "plain"):
            _run_expz_case(c, "c64", path, 9, seed=1)


# ------------------------------------------------------------------ workloads
def _oracle_workload(w, rows=None):
    """Oracle outputs of a workload, for all rows or a sampled subset."""
    idx = np.arange(w.batch) if rows is None else np.asarray(rows)
    feats = None if w.feats is None else w.feats[idx]
    if w.encoding == "amplitude":
        psi0 = O.encode_amplitude(w.x[idx], w.n_qubits)
    else:
        psi0 = O.encode_zero(len(idx), w.n_qubits)
    return idx, feats, psi0


@pytest.mark.parametrize("key,B", [("c1", 64), ("c2", 37), ("c3", 75)])
def test_workload_step_vs_oracle(key, B):
    w = Dt.make_workload(key, B)
    _announce(f"workload {key} B={B}")
    # the separate forward, loss and adjoint launches (the one-launch step
    # has tests of its own)
    d = sim.to_device(w, one_launch=False)
    out = sim.step(d)
    torch.cuda.synchronize()
    idx, feats, psi0 = _oracle_workload(w)
    z = O.expz(O.run_circuit(w.circuit, w.params, feats, psi0))
    tol = TOL[w.dtype]
    np.testing.assert_allclose(out["expz"].cpu().numpy(), z, atol=tol["z"])
    if w.loss == "none":
        return
    L, dz = O.loss_and_dexpz(w.loss, z, w.labels, w.weights)
    assert abs(float(out["loss"]) - L) < tol["z"] * 4
    gth, _ = O.adjoint_vjp(w.circuit, w.params, feats, psi0, dexpz=dz)
    gp, gf = O.theta_to_param_grads(w.circuit, w.params, feats, gth)
    np.testing.assert_allclose(out["grad_params"].cpu().numpy(), gp, atol=tol["grad"])
    if feats is not None:
        np.testing.assert_allclose(out["grad_feats"].cpu().numpy(), gf, atol=tol["grad"])


@pytest.mark.parametrize("key,B", [("c2", 9), ("c3", 11)])
def test_workload_step_c128_vs_oracle(key, B):
    """The complex64 workloads run in complex128 end to end (the same seeded
    inputs), matching the oracle to the FP64 tolerance."""
    w = dataclasses.replace(Dt.make_workload(key, B), dtype="c128")
    _announce(f"workload {key} B={B} c128")
    d = sim.to_device(w)
    out = sim.step(d)
    torch.cuda.synchronize()
    idx, feats, psi0 = _oracle_workload(w)
    z = O.expz(O.run_circuit(w.circuit, w.params, feats, psi0))
    np.testing.assert_allclose(out["expz"].cpu().numpy(), z, atol=1e-10)
    L, dz = O.loss_and_dexpz(w.loss, z, w.labels, w.weights)
    gth, _ = O.adjoint_vjp(w.circuit, w.params, feats, psi0, dexpz=dz)
    gp, gf = O.theta_to_param_grads(w.circuit, w.params, feats, gth)
    np.testing.assert_allclose(out["grad_params"].cpu().numpy(), gp, atol=1e-10)
    if feats is not None:
        np.testing.assert_allclose(out["grad_feats"].cpu().numpy(), gf, atol=1e-10)


def test_autoencoder_step_c128_vs_oracle():
    w = dataclasses.replace(Dt.make_workload("c4", 3), dtype="c128")
    _announce("workload c4 B=3 c128")
    d = sim.to_device(w)
    out = sim.step(d)
    torch.cuda.synchronize()
    F, gth, gph = _fidelity_oracle(w, None, w.batch)
    np.testing.assert_allclose(out["fid"].cpu().numpy(), F, atol=1e-10)
    np.testing.assert_allclose(out["grad_params"].cpu().numpy(), gth, atol=1e-10)
    np.testing.assert_allclose(out["grad_params_dec"].cpu().numpy(), gph, atol=1e-10)


def _fidelity_oracle(w, rows, B_total):
    idx, _, x = _oracle_workload(w, rows)
    psi = O.run_circuit(w.circuit, w.params, None, x)
    chi = O.run_circuit(w.decoder, w.params_dec, None, x)
    dF = -np.ones(len(idx)) / B_total
    if w.loss == "fidelity_trajectory":
        u = Dt.trajectory_uniforms(w.batch)[idx]
        F, m, c, p = O.fidelity_trajectory(psi, chi, w.n_trash, u)
        lam, mu = O.trajectory_fidelity_cotangents(psi, chi, m, c, p, dF, w.n_trash)
    elif w.loss == "fidelity_postselect":
        F, c, p = O.fidelity_postselect(psi, chi, w.n_trash)
        lam, mu = O.postselect_fidelity_cotangents(psi, chi, c, p, dF, w.n_trash)
    else:
        F, cm = O.fidelity_reset(psi, chi, w.n_trash)
        lam, mu = O.reset_channel_fidelity_cotangents(psi, chi, cm, dF, w.n_trash)
    g1, _ = O.adjoint_vjp(w.circuit, w.params, None, x, lam_final=lam)
    g2, _ = O.adjoint_vjp(w.decoder, w.params_dec, None, x, lam_final=mu)
    return F, O.theta_to_param_grads(w.circuit, w.params, None, g1)[0], \
        O.theta_to_param_grads(w.decoder, w.params_dec, None, g2)[0]


def test_autoencoder_step_vs_oracle():
    w = Dt.make_workload("c4", 5)
    _announce("workload c4 B=5")
    d = sim.to_device(w)
    out = sim.step(d)
    torch.cuda.synchronize()
    F, gth, gph = _fidelity_oracle(w, None, w.batch)
    np.testing.assert_allclose(out["fid"].cpu().numpy(), F, atol=1e-5)
    np.testing.assert_allclose(out["grad_params"].cpu().numpy(), gth, atol=1e-4)
    np.testing.assert_allclose(out["grad_params_dec"].cpu().numpy(), gph, atol=1e-4)


@pytest.mark.parametrize("dtype,B", [("c64", 5), ("c128", 3)])
def test_autoencoder_postselect_step_vs_oracle(dtype, B):
    w = dataclasses.replace(Dt.make_workload("c4", B), dtype=dtype,
                            loss="fidelity_postselect")
    _announce(f"workload c4 post-selected B={B} {dtype}")
    d = sim.to_device(w)
    out = sim.step(d)
    torch.cuda.synchronize()
    F, gth, gph = _fidelity_oracle(w, None, w.batch)
    tol = TOL[dtype]
    np.testing.assert_allclose(out["fid"].cpu().numpy(), F, atol=tol["z"])
    np.testing.assert_allclose(float(out["loss"]), 1.0 - F.mean(), atol=tol["z"])
    np.testing.assert_allclose(out["grad_params"].cpu().numpy(), gth, atol=tol["grad"])
    np.testing.assert_allclose(out["grad_params_dec"].cpu().numpy(), gph, atol=tol["grad"])


@pytest.mark.parametrize("dtype,B", [("c64", 5), ("c128", 3)])
def test_autoencoder_trajectory_step_vs_oracle(dtype, B):
    w = dataclasses.replace(Dt.make_workload("c4", B), dtype=dtype,
                            loss="fidelity_trajectory")
    _announce(f"workload c4 trajectory B={B} {dtype}")
    d = sim.to_device(w, traj_u=Dt.trajectory_uniforms(B))
    out = sim.step(d)
    torch.cuda.synchronize()
    F, gth, gph = _fidelity_oracle(w, None, w.batch)
    tol = TOL[dtype]
    np.testing.assert_allclose(out["fid"].cpu().numpy(), F, atol=tol["z"])
    np.testing.assert_allclose(out["grad_params"].cpu().numpy(), gth, atol=tol["grad"])
    np.testing.assert_allclose(out["grad_params_dec"].cpu().numpy(), gph, atol=tol["grad"])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,t,B", [(1, 0, 3), (4, 2, 9), (7, 6, 5), (10, 3, 40), (12, 4, 6),
                                   (15, 1, 2), (3, 1, 0)])
def test_trajectory_fidelity_kernel_vs_oracle(dtype, n, t, B):
    """The kernel alone on seeded random (unnormalised) states with some
    empty slices and one all-zero row: the drawn outcome (exact; the uniforms
    sit mid-interval of a seeded target outcome, away from any boundary), F,
    and both cotangents element by element."""
    _announce(f"trajectory fidelity kernel n={n} t={t} B={B} {dtype}")
    rng = np.random.default_rng(2000 + 37 * n + t)
    N_, M, K = 1 << n, 1 << t, 1 << (n - t)
    cd = torch.complex64 if dtype == "c64" else torch.complex128
    qd = N.QS_C64 if dtype == "c64" else N.QS_C128
    psi = (rng.standard_normal((B, N_)) + 1j * rng.standard_normal((B, N_))) * 0.6
    chi = rng.standard_normal((B, N_)) + 1j * rng.standard_normal((B, N_))
    if B > 1 and M > 1:
        psi[0, K:2 * K] = 0          # outcome 1 impossible in row 0
    if B > 2:
        psi[2] = 0                   # nothing at all: NaN, outcome 0
    P = torch.as_tensor(psi).to("cuda", cd).contiguous()
    X = torch.as_tensor(chi).to("cuda", cd).contiguous()
    psi_r, chi_r = P.cpu().numpy().astype(np.complex128), X.cpu().numpy().astype(np.complex128)
    pm = np.sum(np.abs(psi_r.reshape(B, M, K)) ** 2, axis=2)
    u = np.zeros(B)
    for b in range(B):
        ok_m = np.nonzero(pm[b] > 0)[0]
        if len(ok_m) == 0:
            u[b] = 0.5
            continue
        m = int(rng.choice(ok_m))
        cum = np.cumsum(pm[b]) / pm[b].sum()
        u[b] = ((cum[m - 1] if m > 0 else 0.0) + cum[m]) / 2
    dF = rng.uniform(-1, 1, B)
    fid = torch.full((B,), 7.0, dtype=torch.float64, device="cuda")
    out_m = torch.full((B,), -5, dtype=torch.int32, device="cuda")
    lp = torch.full_like(P, 3.0)
    lc = torch.full_like(P, 3.0)
    N.qs_fidelity_trajectory(qd, n, t, P, X, _dev(u, torch.float64), fid, out_m,
                             _dev(dF, torch.float64), lp, lc)
    torch.cuda.synchronize()
    if B == 0:
        return
    F, m, c, p = O.fidelity_trajectory(psi_r, chi_r, t, u)
    np.testing.assert_array_equal(out_m.cpu().numpy(), m)
    ok = p > 0
    f = fid.cpu().numpy()
    assert np.all(np.isnan(f[~ok]))
    rt = 1e-5 if dtype == "c64" else 1e-12
    np.testing.assert_allclose(f[ok], F[ok], rtol=rt, atol=rt)
    with np.errstate(invalid="ignore", divide="ignore"):
        lam, mu = O.trajectory_fidelity_cotangents(psi_r, chi_r, m, c, p, dF, t)
    scale = np.abs(lam[ok]).max() + np.abs(mu[ok]).max()
    np.testing.assert_allclose(lp.cpu().numpy()[ok], lam[ok], atol=rt * scale, rtol=0)
    np.testing.assert_allclose(lc.cpu().numpy()[ok], mu[ok], atol=rt * scale, rtol=0)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,t,B", [(1, 0, 3), (5, 0, 4), (6, 5, 7), (9, 3, 33), (12, 4, 10),
                                   (15, 2, 2), (3, 1, 0)])
def test_postselect_fidelity_kernel_vs_oracle(dtype, n, t, B):
    """The kernel alone on seeded random (unnormalised) states: F', both
    cotangents element by element, a row where the kept outcome has zero
    probability (NaN there, the other rows untouched), and B = 0."""
    _announce(f"post-selected fidelity kernel n={n} t={t} B={B} {dtype}")
    rng = np.random.default_rng(1000 + 37 * n + t)
    N_ = 1 << n
    cd = torch.complex64 if dtype == "c64" else torch.complex128
    qd = N.QS_C64 if dtype == "c64" else N.QS_C128
    psi = (rng.standard_normal((B, N_)) + 1j * rng.standard_normal((B, N_))) * 0.7
    chi = rng.standard_normal((B, N_)) + 1j * rng.standard_normal((B, N_))
    if B > 1:
        psi[1, :N_ >> t] = 0                       # post-selection impossible
    P = torch.as_tensor(psi).to("cuda", cd).contiguous()
    X = torch.as_tensor(chi).to("cuda", cd).contiguous()
    psi_r, chi_r = P.cpu().numpy().astype(np.complex128), X.cpu().numpy().astype(np.complex128)
    dF = rng.uniform(-1, 1, B)
    fid = torch.full((B,), 7.0, dtype=torch.float64, device="cuda")
    lp = torch.full_like(P, 3.0)
    lc = torch.full_like(P, 3.0)
    N.qs_fidelity_postselect(qd, n, t, P, X, fid, _dev(dF, torch.float64), lp, lc)
    torch.cuda.synchronize()
    if B == 0:
        return
    F, c, p = O.fidelity_postselect(psi_r, chi_r, t)
    with np.errstate(invalid="ignore", divide="ignore"):
        lam, mu = O.postselect_fidelity_cotangents(psi_r, chi_r, c, p, dF, t)
    ok = p > 0
    f = fid.cpu().numpy()
    assert np.all(np.isnan(f[~ok]))
    # inputs are not normalised: compare relative to the size of each quantity
    rt = 1e-5 if dtype == "c64" else 1e-12
    np.testing.assert_allclose(f[ok], F[ok], rtol=rt, atol=rt)
    scale = np.abs(lam[ok]).max() + np.abs(mu[ok]).max()
    np.testing.assert_allclose(lp.cpu().numpy()[ok], lam[ok], atol=rt * scale, rtol=0)
    np.testing.assert_allclose(lc.cpu().numpy()[ok], mu[ok], atol=rt * scale, rtol=0)


def test_full_size_autoencoder_postselect_sampled_rows():
    w = dataclasses.replace(Dt.make_workload("c4"), loss="fidelity_postselect")
    _announce(f"full-size c4 post-selected B={w.batch}")
    rows = np.array([0, 5, 700, 1023])
    d = sim.to_device(w)
    s, sd = d.sim, d.sim_dec
    s.encode_amplitude(d.x, out=d.state)
    sd.encode_amplitude(d.x, out=d.state_dec)
    s.forward(d.params, None, d.state, want_expz=False)
    sd.forward(d.params_dec, None, d.state_dec, want_expz=False)
    B = w.batch
    fid = torch.empty(B, dtype=torch.float64, device="cuda")
    dfid = torch.zeros(B, dtype=torch.float64, device="cuda")
    dfid[rows] = -1.0 / B
    lp, lc = torch.empty_like(d.state), torch.empty_like(d.state)
    N.qs_fidelity_postselect(s.qs_dtype, s.n, w.n_trash, d.state, d.state_dec, fid,
                             dfid, lp, lc)
    g1, _ = s.adjoint(d.params, None, d.state, dstate=lp, ws=d.ws)
    g2, _ = sd.adjoint(d.params_dec, None, d.state_dec, dstate=lc, ws=d.ws_dec)
    torch.cuda.synchronize()
    F, gth, gph = _fidelity_oracle(w, rows, B)
    np.testing.assert_allclose(fid.cpu().numpy()[rows], F, atol=1e-5)
    f_all = fid.cpu().numpy()
    assert np.all((f_all >= -1e-6) & (f_all <= 1 + 1e-6))
    np.testing.assert_allclose(g1.cpu().numpy(), gth, atol=1e-4)
    np.testing.assert_allclose(g2.cpu().numpy(), gph, atol=1e-4)


# ------------------------------------------------- full sizes, sampled rows
def _masked_step(w, rows):
    """GPU forward over the full batch (the launch shape the benchmark times);
    adjoint with the upstream gradient kept only on ``rows``."""
    d = sim.to_device(w)
    s = d.sim
    if w.encoding == "amplitude":
        s.encode_amplitude(d.x, out=d.state)
    else:
        s.zero_state(w.batch, out=d.state)
    z = s.forward(d.params, d.feats, d.state)
    zr = z[rows]
    dz = torch.zeros_like(z)
    L, dzr = O.loss_and_dexpz(w.loss, zr.cpu().numpy(),
                              None if w.labels is None else w.labels[rows],
                              w.weights)
    # loss over the sampled rows only: mean over len(rows)
    dz[rows] = torch.as_tensor(dzr, device="cuda")
    gp, gf = s.adjoint(d.params, d.feats, d.state, dexpz=dz, ws=d.ws)
    torch.cuda.synchronize()
    return z.cpu().numpy(), gp.cpu().numpy(), None if gf is None else gf.cpu().numpy()


@pytest.mark.parametrize("key", ["c2", "c3"])
def test_full_size_sampled_rows(key):
    w = Dt.make_workload(key)
    _announce(f"full-size {key} B={w.batch}")
    rows = np.unique(np.r_[0, 1, w.batch - 1, np.random.default_rng(7).integers(0, w.batch, 5)])
    z, gp, gf = _masked_step(w, rows)
    idx, feats, psi0 = _oracle_workload(w, rows)
    zo = O.expz(O.run_circuit(w.circuit, w.params, feats, psi0))
    np.testing.assert_allclose(z[rows], zo, atol=1e-5)
    assert np.all(np.abs(z) <= 1 + 1e-5)
    _, dz = O.loss_and_dexpz(w.loss, zo, None if w.labels is None else w.labels[rows],
                             w.weights)
    gth, _ = O.adjoint_vjp(w.circuit, w.params, feats, psi0, dexpz=dz)
    rp, rf = O.theta_to_param_grads(w.circuit, w.params, feats, gth)
    np.testing.assert_allclose(gp, rp, atol=1e-4)
    if rf is not None:
        np.testing.assert_allclose(gf[rows], rf, atol=1e-4)
        others = np.setdiff1d(np.arange(w.batch), rows)
        assert np.all(gf[others] == 0)


def test_full_size_autoencoder_sampled_rows():
    w = Dt.make_workload("c4")
    _announce(f"full-size c4 B={w.batch}")
    rows = np.array([0, 3, 511, 1023])
    d = sim.to_device(w)
    s, sd = d.sim, d.sim_dec
    s.encode_amplitude(d.x, out=d.state)
    sd.encode_amplitude(d.x, out=d.state_dec)
    s.forward(d.params, None, d.state, want_expz=False)
    sd.forward(d.params_dec, None, d.state_dec, want_expz=False)
    B = w.batch
    fid = torch.empty(B, dtype=torch.float64, device="cuda")
    dfid = torch.zeros(B, dtype=torch.float64, device="cuda")
    dfid[rows] = -1.0 / B
    lp, lc = torch.empty_like(d.state), torch.empty_like(d.state)
    N.qs_fidelity_reset(s.qs_dtype, s.n, w.n_trash, d.state, d.state_dec, fid,
                        dfid, lp, lc)
    g1, _ = s.adjoint(d.params, None, d.state, dstate=lp, ws=d.ws)
    g2, _ = sd.adjoint(d.params_dec, None, d.state_dec, dstate=lc, ws=d.ws_dec)
    torch.cuda.synchronize()
    F, gth, gph = _fidelity_oracle(w, rows, B)
    np.testing.assert_allclose(fid.cpu().numpy()[rows], F, atol=1e-5)
    f_all = fid.cpu().numpy()
    assert np.all((f_all >= -1e-6) & (f_all <= 1 + 1e-6))
    np.testing.assert_allclose(g1.cpu().numpy(), gth, atol=1e-4)
    np.testing.assert_allclose(g2.cpu().numpy(), gph, atol=1e-4)


# ------------------------------------------- LDS staging, one component a time
@pytest.fixture
def half_staging(monkeypatch):
    monkeypatch.setenv("QS_FWD_HALF_STAGING", "1")
    monkeypatch.setenv("QS_ADJ_HALF_STAGING", "1")


@pytest.mark.parametrize("n", [1, 3, 6, 10, 13, 14])
def test_half_staging_random_circuits(n, half_staging, monkeypatch):
    rng = np.random.default_rng(900 + n)
    c = C.random_circuit(n, 80, rng, n_params=7, n_features=3)
    half = sim.Simulator(c, "c64").plan_info(5)
    monkeypatch.delenv("QS_FWD_HALF_STAGING")
    full = sim.Simulator(c, "c64").plan_info(5)
    monkeypatch.setenv("QS_FWD_HALF_STAGING", "1")
    # the same samples per block need less LDS with one component staged
    per_sample = (full["lds_bytes"] / full["samples_per_block"],
                  half["lds_bytes"] / half["samples_per_block"])
    assert per_sample[1] < per_sample[0]
    _run_expz_case(c, "c64", "fused", 33 if n <= 10 else 3, seed=n)


@pytest.mark.parametrize("kind", ["start_end", "zz", "cancel"])
def test_half_staging_cnot_patterns_and_per_sample(kind, half_staging):
    _run_expz_case(cnot_pattern(9, kind), "c64", "fused", 21, seed=6)
    rng = np.random.default_rng(33)
    c = C.random_circuit(8, 60, rng, n_params=6, n_features=2)
    _run_expz_case(c, "c64", "fused", 19, seed=7, per_sample=True)
    _run_expz_case(c, "c64", "fused", 13, seed=8, dstate_mode=True, amplitude=False)


def test_half_staging_full_size_c3_sampled_rows(half_staging):
    test_full_size_sampled_rows("c3")


# ----------------------------------------------------------------- edge cases
def test_zero_norm_rows_are_counted_and_nan():
    c = C.hea_ry_rz_ring(3, 1)
    s = sim.Simulator(c, "c64")
    x = torch.randn(4, 8, device="cuda")
    x[2] = 0
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = s.empty_state(4)
    N.qs_encode(N.QS_ENC_AMPLITUDE, s.qs_dtype, 3, x, st, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 1
    assert torch.isnan(st[2].real).all()
    assert torch.isfinite(st[[0, 1, 3]].real).all()


@pytest.mark.parametrize("dtype,xbits", [("c64", 32), ("c128", 64), ("c64", 64)])
@pytest.mark.parametrize("n", [1, 3, 5, 8, 10, 12, 13, 14])
def test_forward_amplitude_vs_oracle(n, dtype, xbits):
    """Encoding fused into the engine's state load (x in the state's
    precision) and the encode-then-forward fallback (x in the other one):
    final states and <Z> against the oracle, on a zero-padded input read
    through a row stride wider than D, with one zero row that must come out
    NaN and be counted; other rows are unaffected by it."""
    rng = np.random.default_rng(1500 + n)
    c = C.random_circuit(n, 60, rng, n_params=6, n_features=2)
    B = 13 if n <= 10 else 3
    _announce(f"forward_amplitude n={n} {dtype} x{xbits} B={B}")
    rd = np.float32 if xbits == 32 else np.float64
    D = max(1, (1 << n) - (1 << n) // 5)
    wide = rng.standard_normal((B, D + 3)).astype(rd)
    zero_row = B // 2
    wide[zero_row] = 0
    s = sim.Simulator(c, dtype, PATHS["auto"])
    params = rng.uniform(-np.pi, np.pi, c.n_params)
    feats = rng.uniform(-1, 1, (B, c.n_features))
    pt, ft = _dev(params, s.rdtype), _dev(feats, s.rdtype)
    xt = _dev(wide, torch.float32 if xbits == 32 else torch.float64)[:, :D]
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = s.empty_state(B)
    z = s.forward(pt, ft, st, x=xt, bad_rows=bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 1
    assert torch.isnan(st[zero_row].real).all() and torch.isnan(st[zero_row].imag).all()
    keep = [b for b in range(B) if b != zero_row]
    x_used = wide[keep, :D].astype(np.float64)
    psi0 = O.encode_amplitude(x_used, n)
    rn = np.float32 if dtype == "c64" else np.float64  # what the GPU was given
    pc = params.astype(rn).astype(np.float64)
    fc = feats[keep].astype(rn).astype(np.float64)
    psiG = O.run_circuit(c, pc, fc, psi0)
    tol = TOL[dtype]
    np.testing.assert_allclose(st.cpu().numpy()[keep], psiG, atol=tol["state"])
    np.testing.assert_allclose(z.cpu().numpy()[keep], O.expz(psiG), atol=tol["z"])


@pytest.mark.parametrize("n", [4, 10, 13])
def test_forward_amplitude_with_one_component_staging(n, half_staging):
    """Launches that stage one state component at a time get an encoded
    state (the encoding kernel, then the sweep) instead of encoding while
    they load: the same results."""
    test_forward_amplitude_vs_oracle(n, "c64", 32)


def test_forward_amplitude_with_checkpoints_matches_encode_then_forward():
    """With checkpoints the fused forward stores the same states as qs_encode
    followed by qs_forward, and ends in the same final state."""
    rng = np.random.default_rng(1600)
    c = C.hea_ry_rz_ring(9, 6)
    B = 33
    s = sim.Simulator(c, "c64", PATHS["fused"])
    pt = _dev(rng.uniform(-np.pi, np.pi, c.n_params), torch.float32)
    xt = _dev(rng.standard_normal((B, 512)), torch.float32)
    ck_g = [c.layer_end[1], c.layer_end[3]]
    ck_a = torch.empty((2, B, 512), dtype=torch.complex64, device="cuda")
    ck_b = torch.empty_like(ck_a)
    st_a = s.empty_state(B)
    za = s.forward(pt, None, st_a, ckpt_gates=ck_g, ckpt=ck_a, x=xt)
    st_b = s.encode_amplitude(xt)
    zb = s.forward(pt, None, st_b, ckpt_gates=ck_g, ckpt=ck_b)
    torch.cuda.synchronize()
    for a, b in ((st_a, st_b), (ck_a, ck_b), (za, zb)):
        np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), atol=2e-6)


def _train_case(c, B, seed, q, amplitude, dtype="c64"):
    """qs_train_step_mse against the oracle and against the three calls it
    fuses (forward from the encoding, loss kernel, adjoint)."""
    rng = np.random.default_rng(seed)
    n = c.n_qubits
    s = sim.Simulator(c, dtype)
    need = N.qs_train_workspace_size(s.h, s.qs_dtype, B)
    assert need > 0, "the one-launch training step should run for this shape"
    params = rng.uniform(-np.pi, np.pi, c.n_params).astype(np.float32)
    feats = rng.uniform(-1, 1, (B, c.n_features)).astype(np.float32) if c.n_features else None
    y = rng.choice([-1.0, 1.0], B)
    pt, ft, yt = _dev(params, torch.float32), _dev(feats, torch.float32), _dev(y, torch.float64)
    if amplitude:
        D = max(1, (1 << n) - (1 << n) // 4)
        x = rng.standard_normal((B, D)).astype(np.float32)
        xt = _dev(x, torch.float32)
        psi0 = O.encode_amplitude(x.astype(np.float64), n)
    else:
        xt = None
        psi0 = O.encode_zero(B, n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    z = torch.empty((B, n), dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    gp = torch.empty(c.n_params, dtype=torch.float64, device="cuda")
    gf = torch.empty((B, c.n_features), dtype=torch.float64, device="cuda") if c.n_features else None
    N.qs_train_step_mse(s.h, s.qs_dtype, pt, ft, xt, yt, q, loss, gp, ws, expz=z,
                        grad_feats=gf, B=B)
    torch.cuda.synchronize()
    pc = params.astype(np.float64)
    fc = None if feats is None else feats.astype(np.float64)
    zo = O.expz(O.run_circuit(c, pc, fc, psi0))
    r = zo[:, q] - y
    dz = np.zeros((B, n))
    dz[:, q] = 2.0 * r / B
    gth, _ = O.adjoint_vjp(c, pc, fc, psi0, dexpz=dz)
    rp, rf = O.theta_to_param_grads(c, pc, fc, gth)
    tol = TOL[dtype]
    np.testing.assert_allclose(z.cpu().numpy(), zo, atol=tol["z"])
    assert abs(float(loss.item()) - float(np.mean(r * r))) < 4 * tol["z"]
    np.testing.assert_allclose(gp.cpu().numpy(), rp, atol=tol["grad"])
    if gf is not None:
        np.testing.assert_allclose(gf.cpu().numpy(), rf, atol=tol["grad"])
    # the three separate calls give the same numbers up to rounding order
    st = s.empty_state(B)
    if xt is None:
        s.zero_state(B, out=st)
    z2 = s.forward(pt, ft, st, x=xt)
    dz2 = torch.empty_like(z2)
    loss2 = torch.empty(1, dtype=torch.float64, device="cuda")
    N.qs_loss_mse_z(q, z2, yt, dexpz=dz2, loss=loss2)
    gp2, gf2 = s.adjoint(pt, ft, st, dexpz=dz2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(z.cpu().numpy(), z2.cpu().numpy(), atol=1e-6)
    assert abs(float(loss.item()) - float(loss2.item())) < 1e-6
    np.testing.assert_allclose(gp.cpu().numpy(), gp2.cpu().numpy(), atol=2e-5)


@pytest.mark.parametrize("n,B,q,amp", [(10, 37, 0, True), (4, 300, 3, True), (6, 65, 2, False),
                                       (9, 21, 8, True), (12, 5, 5, True), (13, 3, 0, False)])
def test_train_step_random_circuits(n, B, q, amp):
    rng = np.random.default_rng(2000 + n)
    c = C.random_circuit(n, 70, rng, n_params=6, n_features=2)
    _announce(f"train step n={n} B={B} q={q} amplitude={amp}")
    _train_case(c, B, 2100 + n, q, amp)


@pytest.mark.parametrize("nf", [4, 6])
def test_train_step_feature_counts(nf):
    """The one-launch step with feature gradients in registers (four
    features) and in LDS sums (six)."""
    rng = np.random.default_rng(2400 + nf)
    c = C.random_circuit(9, 60, rng, n_params=6, n_features=nf)
    _announce(f"train step features={nf}")
    _train_case(c, 29, 2500 + nf, 1, True)


@pytest.mark.parametrize("key,B", [("c2", 37), ("c2", 4096)])
def test_train_step_workloads(key, B):
    """The headline circuit's step (10 qubits, amplitude inputs, MSE on
    qubit 0), through sim.step's default path (one launch), against the
    oracle on sampled rows."""
    w = Dt.make_workload(key, B)
    _announce(f"train step workload {key} B={B}")
    d = sim.to_device(w)
    assert sim.train_step_runs(d)
    out = sim.step(d)
    torch.cuda.synchronize()
    rows = np.arange(B) if B <= 64 else np.random.default_rng(5).choice(B, 48, replace=False)
    idx, feats, psi0 = _oracle_workload(w, rows)
    z = O.expz(O.run_circuit(w.circuit, w.params, feats, psi0))
    np.testing.assert_allclose(out["expz"].cpu().numpy()[idx], z, atol=1e-5)
    if B <= 64:
        L, dz = O.loss_and_dexpz(w.loss, z, w.labels, w.weights)
        assert abs(float(out["loss"]) - L) < 4e-5
        gth, _ = O.adjoint_vjp(w.circuit, w.params, feats, psi0, dexpz=dz)
        gp, _ = O.theta_to_param_grads(w.circuit, w.params, feats, gth)
        np.testing.assert_allclose(out["grad_params"].cpu().numpy(), gp, atol=1e-4)


def test_train_step_refuses_what_it_does_not_run(monkeypatch):
    """Per-sample parameters, complex128, float64 inputs and shapes staging
    one component at a time have no one-launch kernel: workspace size 0 and
    QS_ERR_UNSUPPORTED, nothing launched."""
    c = C.hea_ry_rz_ring(6, 2)
    h = N.CircuitHandle(c)
    assert N.qs_train_workspace_size(h, N.QS_C64, 8) > 0
    assert N.qs_train_workspace_size(h, N.QS_C128, 8) == 0
    assert N.qs_train_workspace_size(h, N.QS_C64, 8, N.QS_FLAG_PER_SAMPLE_PARAMS) == 0
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    p = torch.zeros(c.n_params, device="cuda")
    y = torch.zeros(8, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    gp = torch.empty(c.n_params, dtype=torch.float64, device="cuda")
    x64 = torch.ones((8, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(N.QsError) as e:
        N.qs_train_step_mse(h, N.QS_C64, p, None, x64, y, 0, loss, gp, ws)
    assert e.value.status == N.QS_ERR_UNSUPPORTED
    with pytest.raises(N.QsError) as e:
        N.qs_train_step_mse(h, N.QS_C128, p.double(), None, None, y, 0, loss, gp, ws, B=8)
    assert e.value.status == N.QS_ERR_UNSUPPORTED
    monkeypatch.setenv("QS_ADJ_HALF_STAGING", "1")  # the adjoint's shape stages one component
    assert N.qs_train_workspace_size(h, N.QS_C64, 8) == 0


@pytest.mark.parametrize("B,n,q", [(1, 1, 0), (37, 10, 0), (4096, 10, 0), (777, 8, 7),
                                   (65536, 8, 0), (0, 3, 1)])
def test_loss_mse_z(B, n, q):
    """The loss kernel's upstream gradient is (2/B)(z - y) in column q and 0
    elsewhere (the same FP64 operations as written here, so bit for bit);
    its loss is the mean squared residual, summed in a fixed order."""
    rng = np.random.default_rng(1700 + B)
    z = rng.uniform(-1, 1, (B, n))
    y = rng.choice([-1.0, 1.0], B)
    zt, yt = _dev(z, torch.float64), _dev(y, torch.float64)
    dz = torch.full((B, n), 7.0, dtype=torch.float64, device="cuda")
    loss = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    N.qs_loss_mse_z(q, zt, yt, dexpz=dz, loss=loss)
    torch.cuda.synchronize()
    want = np.zeros((B, n))
    if B:
        want[:, q] = 2.0 * (1.0 / B) * (z[:, q] - y)
    np.testing.assert_array_equal(dz.cpu().numpy(), want)
    ref = float(np.mean((z[:, q] - y) ** 2)) if B else 0.0
    assert abs(float(loss.item()) - ref) <= 1e-13 * max(1.0, ref)
    # bitwise reproducible from call to call
    loss2 = torch.zeros_like(loss)
    N.qs_loss_mse_z(q, zt, yt, loss=loss2)
    torch.cuda.synchronize()
    assert float(loss2.item()) == float(loss.item())


def test_encode_check_reports_zero_norm_rows():
    """The counter of zero-norm rows becomes a host-visible status."""
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = torch.empty(3, 8, dtype=torch.complex64, device="cuda")
    x = torch.randn(3, 8, device="cuda")
    N.qs_encode(N.QS_ENC_AMPLITUDE, N.QS_C64, 3, x, st, bad)
    N.qs_encode_check(bad)  # no zero row: no error
    x[1] = 0
    N.qs_encode(N.QS_ENC_AMPLITUDE, N.QS_C64, 3, x, st, bad)
    with pytest.raises(N.QsError) as e:
        N.qs_encode_check(bad)
    assert e.value.status == N.QS_ERR_ZERO_NORM
    assert int(bad.item()) == 1


@pytest.mark.parametrize("path", ["fused", "hbm"])
def test_first_call_inside_a_capture_returns_a_status_and_keeps_the_capture(path):
    """A shape with no plan yet inside a stream capture: the call returns
    QS_ERR_CAPTURE without enqueueing anything, the capture ends normally and
    its graph replays; outside the capture the same call plans and runs."""
    n = 7 if path == "fused" else 15
    c = C.hea_ry_rz_ring(n, 3)
    # a parameter layout no other test uses, so this shape is not planned yet
    c.gates["scale"] = np.where(np.isin(c.gates["op"], list(C.ROTATIONS)), 0.731, 1.0)
    s = sim.Simulator(c, "c64", 0 if path == "fused" else PATHS["hbm"])
    p = torch.full((c.n_params,), 0.3, device="cuda")
    st = s.zero_state(2)
    out = torch.zeros(2, n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        with pytest.raises(N.QsError) as e:
            N.qs_forward(s.h, s.qs_dtype, p, None, st, out)
        out.add_(1.0)
    assert e.value.status == N.QS_ERR_CAPTURE
    g.replay()
    torch.cuda.synchronize()
    assert torch.all(out == 1.0)
    z = s.forward(p, None, st)  # plans outside the capture
    torch.cuda.synchronize()
    ref = O.expz(O.run_circuit(c, np.full(c.n_params, 0.3), None, O.encode_zero(2, n)))
    np.testing.assert_allclose(z.cpu().numpy(), ref, atol=1e-5)


def test_zero_batch_is_a_no_op():
    c = C.hea_ry_rz_ring(4, 1)
    for path in (1, 2):
        s = sim.Simulator(c, "c64", path)
        st = s.empty_state(0)
        p = torch.zeros(c.n_params, device="cuda")
        z = s.forward(p, None, st)
        assert z.shape == (0, 4)
        gp, _ = s.adjoint(p, None, st, dexpz=torch.zeros(0, 4, dtype=torch.float64,
                                                          device="cuda"))
        torch.cuda.synchronize()
        assert torch.all(gp == 0)


def test_invalid_calls_raise():
    c = C.hea_ry_rz_ring(3, 1)
    s = sim.Simulator(c, "c64")
    st = s.zero_state(2)
    p = torch.zeros(c.n_params, device="cuda")
    with pytest.raises(N.QsError):
        s.adjoint(p, None, st)  # neither dexpz nor dstate
    with pytest.raises(N.QsError):
        N.qs_adjoint_backward(s.h, s.qs_dtype, p, None, st,
                              dexpz=torch.zeros(2, 3, dtype=torch.float64, device="cuda"),
                              grad_params=torch.zeros(c.n_params, dtype=torch.float64,
                                                      device="cuda"),
                              ws=None)  # workspace missing
    with pytest.raises(N.QsError):
        s.forward(p, None, st, ckpt_gates=[0], ckpt=st)  # checkpoint at 0


@pytest.mark.parametrize("path", ["fused", "plain"])
def test_checkpoints_store_states_and_reanchor(path):
    w = Dt.make_workload("c2", 9)
    c = w.circuit
    ck = c.layer_end[1:-1:2]  # after layers 2, 4, 6
    s = sim.Simulator(c, "c64", PATHS[path])
    x = _dev(w.x, torch.float32)
    st = s.encode_amplitude(x)
    buf = torch.empty((len(ck),) + tuple(st.shape), dtype=st.dtype, device="cuda")
    p = _dev(w.params, torch.float32)
    s.forward(p, None, st, ckpt_gates=ck, ckpt=buf)
    dz = torch.zeros(9, 10, dtype=torch.float64, device="cuda")
    dz[:, 0] = 0.1
    gp, _ = s.adjoint(p, None, st, dexpz=dz, ckpt_gates=ck, ckpt=buf)
    torch.cuda.synchronize()
    psi0 = O.encode_amplitude(w.x, 10)
    for i, g in enumerate(ck):
        sub = C.Circuit(10, c.gates[:g], c.n_params)
        ref = O.run_circuit(sub, w.params, None, psi0)
        np.testing.assert_allclose(buf[i].cpu().numpy(), ref, atol=1e-5)
    gth, _ = O.adjoint_vjp(c, w.params, None, psi0, dexpz=dz.cpu().numpy())
    rp, _ = O.theta_to_param_grads(c, w.params, None, gth)
    np.testing.assert_allclose(gp.cpu().numpy(), rp, atol=1e-4)


# ------------------------------------------------- CNOTs folded into remaps
@pytest.mark.parametrize("kind", ["start_end", "zz", "cancel", "only"])
@pytest.mark.parametrize("n", [3, 7, 11])
def test_cnot_folding_patterns(n, kind):
    rng = np.random.default_rng(700 + n)
    c = cnot_pattern(n, kind)
    _run_expz_case(c, "c64", "fused", 9, seed=n)
    if c.n_params:
        _run_expz_case(c, "c64", "fused", 5, seed=n + 1, per_sample=True)
    if n <= 7:
        _run_expz_case(c, "c128", "fused", 4, seed=n + 2)


def test_cnot_folding_with_checkpoints_after_cnot_runs():
    """Checkpoints placed right after CNOT runs: the stored states are the
    states after those gates, and the backward re-anchors to them."""
    rng = np.random.default_rng(9)
    n = 9
    c = cnot_pattern(n, "start_end")
    ops = c.gates["op"]
    ck = [g + 1 for g in range(c.n_gates - 1)
          if ops[g] == C.OP["CNOT"] and ops[g + 1] != C.OP["CNOT"]]
    B = 6
    params = rng.uniform(-np.pi, np.pi, c.n_params).astype(np.float32)
    x = rng.standard_normal((B, 1 << n)).astype(np.float32)
    s = sim.Simulator(c, "c64", PATHS["fused"])
    st = s.encode_amplitude(_dev(x, torch.float32))
    buf = torch.empty((len(ck),) + tuple(st.shape), dtype=st.dtype, device="cuda")
    p = _dev(params, torch.float32)
    s.forward(p, None, st, ckpt_gates=ck, ckpt=buf)
    dz = torch.as_tensor(rng.uniform(-1, 1, (B, n)), device="cuda")
    gp, _ = s.adjoint(p, None, st, dexpz=dz, ckpt_gates=ck, ckpt=buf)
    torch.cuda.synchronize()
    psi0 = O.encode_amplitude(x, n)
    for i, g in enumerate(ck):
        ref = O.run_circuit(C.Circuit(n, c.gates[:g], c.n_params), params, None, psi0)
        np.testing.assert_allclose(buf[i].cpu().numpy(), ref, atol=1e-5)
    gth, _ = O.adjoint_vjp(c, params, None, psi0, dexpz=dz.cpu().numpy())
    np.testing.assert_allclose(gp.cpu().numpy(),
                               O.theta_to_param_grads(c, params, None, gth)[0], atol=1e-4)


def test_autograd_function_matches_oracle():
    rng = np.random.default_rng(5)
    c = C.random_circuit(5, 40, rng, n_params=6, n_features=2)
    s = sim.Simulator(c, "c64")
    B = 6
    x = rng.standard_normal((B, 32)).astype(np.float32)
    params = torch.tensor(rng.uniform(-3, 3, 6).astype(np.float32), device="cuda",
                          requires_grad=True)
    feats = torch.tensor(rng.uniform(-1, 1, (B, 2)).astype(np.float32), device="cuda",
                         requires_grad=True)
    st0 = s.encode_amplitude(_dev(x, torch.float32))
    z = sim.expz(params, feats, st0, s)
    wts = torch.tensor(rng.uniform(-1, 1, (B, 5)), device="cuda")
    (z * wts).sum().backward()
    psi0 = O.encode_amplitude(x, 5)
    p64 = params.detach().cpu().numpy()
    f64 = feats.detach().cpu().numpy()
    gth, _ = O.adjoint_vjp(c, p64, f64, psi0, dexpz=wts.cpu().numpy())
    rp, rf = O.theta_to_param_grads(c, p64, f64, gth)
    np.testing.assert_allclose(params.grad.cpu().numpy(), rp, atol=1e-4)
    np.testing.assert_allclose(feats.grad.cpu().numpy(), rf, atol=1e-4)


# ------------------------------------------------- mid-circuit channels
def _run_channel_case(c, dtype, B, seed, per_sample=False, dstate_mode=False,
                      extra_ckpt=()):
    """Forward (state, <Z>, the stored states in front of the channels) and
    adjoint of a circuit with RESET / MEASURE gates, against the oracle."""
    _announce(f"channels n={c.n_qubits} G={c.n_gates} B={B} {dtype} ps={per_sample} "
              f"dstate={dstate_mode}")
    rng = np.random.default_rng(seed)
    n = c.n_qubits
    rd = np.float32 if dtype == "c64" else np.float64
    P = c.n_params
    params = rng.uniform(-np.pi, np.pi, (B, P) if per_sample else P).astype(rd)
    x = rng.standard_normal((B, 1 << n)).astype(rd)
    psi0 = O.encode_amplitude(x, n)
    feats = rng.uniform(-1, 1, (B, c.n_features))
    feats = stable_uniforms(c, params, feats, psi0).astype(rd)
    ck = sorted(set(channel_gates(c)) | set(extra_ckpt))
    flags = N.QS_FLAG_PER_SAMPLE_PARAMS if per_sample else 0
    s = sim.Simulator(c, dtype, flags)
    st = s.encode_amplitude(_dev(x, s.rdtype))
    buf = torch.empty((len(ck),) + tuple(st.shape), dtype=st.dtype, device="cuda")
    pt, ft = _dev(params, s.rdtype), _dev(feats, s.rdtype)
    z = s.forward(pt, ft, st, ckpt_gates=ck, ckpt=buf)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    psiG = O.run_circuit(c, params, feats, psi0)
    np.testing.assert_allclose(st.cpu().numpy(), psiG, atol=tol["state"])
    np.testing.assert_allclose(z.cpu().numpy(), O.expz(psiG), atol=tol["z"])
    for i, g in enumerate(ck):
        ref = O.run_circuit(C.Circuit(n, c.gates[:g], P, c.n_features), params, feats, psi0)
        np.testing.assert_allclose(buf[i].cpu().numpy(), ref, atol=tol["state"])
    if dstate_mode:
        lam = (rng.standard_normal((B, 1 << n)) + 1j * rng.standard_normal((B, 1 << n))) * 0.3
        gp, gf = s.adjoint(pt, ft, st, dstate=_dev(lam, s.cdtype), ckpt_gates=ck, ckpt=buf)
        gth, _ = O.adjoint_vjp(c, params, feats, psi0, lam_final=lam)
    else:
        dz = rng.uniform(-1, 1, (B, n))
        gp, gf = s.adjoint(pt, ft, st, dexpz=_dev(dz, torch.float64), ckpt_gates=ck, ckpt=buf)
        gth, _ = O.adjoint_vjp(c, params, feats, psi0, dexpz=dz)
    torch.cuda.synchronize()
    rp, rf = O.theta_to_param_grads(c, params, feats, gth)
    np.testing.assert_allclose(gp.cpu().numpy(), rp, atol=tol["grad"])
    np.testing.assert_allclose(gf.cpu().numpy(), rf, atol=tol["grad"])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,G,where", [(1, 12, [3, 8]), (3, 40, [0, 17, 17, 40]),
                                       (6, 80, [25, 50]), (10, 120, [30, 61, 90]),
                                       (13, 90, [44])])
def test_mid_circuit_channels_vs_oracle(n, G, where, dtype):
    """Reset and measurement channels inside random circuits (every gate
    kind, features, shared parameters), including channels at the start, at
    the end and back to back, with extra checkpoints between them: states,
    <Z>, the stored states, parameter and feature gradients."""
    rng = np.random.default_rng(1300 + n)
    c = C.with_channels(C.random_circuit(n, G, rng, n_params=7, n_features=2), where, rng)
    extra = [g + 1 for g in channel_gates(c) if g + 1 < c.n_gates][:1] + [2]
    _run_channel_case(c, dtype, 5, seed=n, extra_ckpt=[e for e in extra if 0 < e < c.n_gates])
    _run_channel_case(c, dtype, 3, seed=n + 1, per_sample=True)
    _run_channel_case(c, dtype, 3, seed=n + 2, dstate_mode=True)


def test_mid_circuit_channel_calls_refuse_what_they_cannot_run():
    rng = np.random.default_rng(1399)
    c = C.with_channels(C.hea_ry_rz_ring(6, 2), [5, 20], rng)
    s = sim.Simulator(c, "c64")
    st = s.zero_state(2)
    p = torch.zeros(c.n_params, device="cuda")
    f = torch.full((2, c.n_features), 0.5, device="cuda")
    ck = channel_gates(c)
    buf = torch.empty((len(ck),) + tuple(st.shape), dtype=st.dtype, device="cuda")
    with pytest.raises(N.QsError) as e:  # no checkpoint in front of the second channel
        s.forward(p, f, st, ckpt_gates=ck[:1], ckpt=buf)
    assert e.value.status == N.QS_ERR_INVALID
    with pytest.raises(N.QsError) as e:  # a channel has no inverse
        s.forward(p, f, st, ckpt_gates=ck, ckpt=buf, flags=N.QS_FLAG_INVERSE)
    assert e.value.status == N.QS_ERR_INVALID
    with pytest.raises(N.QsError) as e:  # gate by gate: not for channels
        s.forward(p, f, st, ckpt_gates=ck, ckpt=buf, flags=N.QS_PATH_PLAIN)
    assert e.value.status == N.QS_ERR_UNSUPPORTED


# ------------------------------------- finite differences on the GPU itself
@pytest.mark.parametrize("key", ["c2", "c3"])
def test_adjoint_matches_gpu_central_differences_c128(key):
    """The complex128 adjoint against central differences of the complex128
    forward, both on the GPU (no oracle in the loop): L = sum_b,q w_bq <Z_q>_b,
    h = 1e-5 on every parameter (and every feature of the re-uploading
    circuit)."""
    w = Dt.make_workload(key, 3)
    c = w.circuit
    _announce(f"GPU central differences {key} c128")
    rng = np.random.default_rng(41)
    s = sim.Simulator(c, "c128")
    B, n = 3, c.n_qubits
    params = torch.tensor(rng.uniform(-np.pi, np.pi, c.n_params), device="cuda")
    feats = (torch.tensor(rng.uniform(-1, 1, (B, c.n_features)), device="cuda")
             if c.n_features else None)
    if w.encoding == "amplitude":
        st0 = s.encode_amplitude(_dev(rng.standard_normal((B, 1 << n)), torch.float64))
    else:
        st0 = s.zero_state(B)
    wts = torch.tensor(rng.uniform(-1, 1, (B, n)), device="cuda")

    def loss(p, f):
        st = st0.clone()
        return float((s.forward(p, f, st) * wts).sum().item())

    st = st0.clone()
    s.forward(params, feats, st, want_expz=False)
    gp, gf = s.adjoint(params, feats, st, dexpz=wts)
    gp = gp.cpu().numpy()
    h = 1e-5
    fd = np.zeros(c.n_params)
    for i in range(c.n_params):
        pp, pm = params.clone(), params.clone()
        pp[i] += h
        pm[i] -= h
        fd[i] = (loss(pp, feats) - loss(pm, feats)) / (2 * h)
    np.testing.assert_allclose(gp, fd, atol=1e-8)
    if feats is not None:
        fdf = np.zeros((B, c.n_features))
        for b in range(B):
            for k in range(c.n_features):
                fp, fm = feats.clone(), feats.clone()
                fp[b, k] += h
                fm[b, k] -= h
                fdf[b, k] = (loss(params, fp) - loss(params, fm)) / (2 * h)
        np.testing.assert_allclose(gf.cpu().numpy(), fdf, atol=1e-8)


def test_autograd_gradcheck_c128():
    """torch.autograd.gradcheck (its own finite differences) through the
    <Z> Function in complex128, parameters and features."""
    rng = np.random.default_rng(43)
    c = C.random_circuit(4, 30, rng, n_params=5, n_features=2)
    s = sim.Simulator(c, "c128")
    st0 = s.encode_amplitude(_dev(rng.standard_normal((2, 16)), torch.float64))
    p = torch.tensor(rng.uniform(-2, 2, 5), device="cuda", requires_grad=True)
    f = torch.tensor(rng.uniform(-1, 1, (2, 2)), device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b: sim.expz(a, b, st0, s), (p, f),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)


def _fidelity_setup(dtype, rng, n=6, t=2, B=4):
    enc = C.ry_rz_chain(n, 3)
    rd = np.float32 if dtype == "c64" else np.float64
    th = rng.uniform(-np.pi, np.pi, enc.n_params).astype(rd)
    ph = rng.uniform(-np.pi, np.pi, enc.n_params).astype(rd)
    x = rng.standard_normal((B, 1 << n)).astype(rd)
    return enc, th, ph, x


@pytest.mark.parametrize("kind", ["reset", "postselect", "trajectory"])
def test_fidelity_autograd_matches_oracle(kind):
    """The fidelity losses through torch.autograd (complex64) against the
    oracle's cotangents and adjoint, and a complex128 gradcheck."""
    rng = np.random.default_rng(47)
    n, t, B = 6, 2, 4
    enc, th, ph, x = _fidelity_setup("c64", rng, n, t, B)
    psi0 = O.encode_amplitude(x, n)
    psi = O.run_circuit(enc, th, None, psi0)
    chi = O.run_circuit(enc, ph, None, psi0)
    u = None
    if kind == "trajectory":  # mid-interval uniforms: the outcome is 1 for every row
        pm = np.abs(psi.reshape(B, 1 << t, -1)) ** 2
        pm = pm.sum(axis=2)
        u = (pm[:, 0] + 0.5 * pm[:, 1]) / pm.sum(axis=1)
    dF = -np.ones(B) / B
    if kind == "reset":
        F, cm = O.fidelity_reset(psi, chi, t)
        lam, mu = O.reset_channel_fidelity_cotangents(psi, chi, cm, dF, t)
    elif kind == "postselect":
        F, cc, pp = O.fidelity_postselect(psi, chi, t)
        lam, mu = O.postselect_fidelity_cotangents(psi, chi, cc, pp, dF, t)
    else:
        F, m, cc, pp = O.fidelity_trajectory(psi, chi, t, u)
        assert np.all(m == 1)
        lam, mu = O.trajectory_fidelity_cotangents(psi, chi, m, cc, pp, dF, t)
    g1, _ = O.adjoint_vjp(enc, th, None, psi0, lam_final=lam)
    g2, _ = O.adjoint_vjp(enc, ph, None, psi0, lam_final=mu)
    ref_th = O.theta_to_param_grads(enc, th, None, g1)[0]
    ref_ph = O.theta_to_param_grads(enc, ph, None, g2)[0]
    se, sd = sim.Simulator(enc, "c64"), sim.Simulator(enc, "c64")
    st0 = se.encode_amplitude(_dev(x, torch.float32))
    pt = torch.tensor(th, device="cuda", requires_grad=True)
    pd = torch.tensor(ph, device="cuda", requires_grad=True)
    ut = None if u is None else _dev(u, torch.float64)
    fid = sim.autoencoder_fidelity(pt, pd, st0, se, sd, t, kind, ut)
    loss = 1.0 - fid.mean()
    loss.backward()
    np.testing.assert_allclose(fid.detach().cpu().numpy(), F, atol=1e-5)
    np.testing.assert_allclose(pt.grad.cpu().numpy(), ref_th, atol=1e-4)
    np.testing.assert_allclose(pd.grad.cpu().numpy(), ref_ph, atol=1e-4)
    # complex128: gradcheck through the same Function
    enc2, th2, ph2, x2 = _fidelity_setup("c128", rng, 5, 1, 2)
    s2e, s2d = sim.Simulator(enc2, "c128"), sim.Simulator(enc2, "c128")
    st2 = s2e.encode_amplitude(_dev(x2, torch.float64))
    u2 = None
    if kind == "trajectory":
        q = np.abs(O.run_circuit(enc2, th2, None, O.encode_amplitude(x2, 5))
                   .reshape(2, 2, -1)) ** 2
        q = q.sum(axis=2)
        u2 = _dev(0.5 * q[:, 0] / q.sum(axis=1), torch.float64)  # outcome 0
    a = torch.tensor(th2, device="cuda", requires_grad=True)
    b = torch.tensor(ph2, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(
        lambda p1, p2: sim.autoencoder_fidelity(p1, p2, st2, s2e, s2d, 1, kind, u2),
        (a, b), eps=1e-6, atol=1e-7, rtol=1e-5)


# ------------------------------------------------ large states: tiled path
@pytest.fixture
def tile_qubits(monkeypatch):
    def set_m(m):
        monkeypatch.setenv("QS_TILE_QUBITS", str(m))
    return set_m


@pytest.mark.parametrize("n,m", [(6, 4), (8, 5), (9, 6), (11, 7)])
def test_tiled_path_random_circuits(n, m, tile_qubits):
    tile_qubits(m)
    rng = np.random.default_rng(500 + n)
    c = C.random_circuit(n, 80, rng, n_params=6, n_features=2)
    _run_expz_case(c, "c64", "hbm", 5, seed=n)
    _run_expz_case(c, "c64", "hbm", 3, seed=n + 1, per_sample=True)
    _run_expz_case(c, "c64", "hbm", 3, seed=n + 2, dstate_mode=True, amplitude=False)


@pytest.mark.parametrize("kind", ["start_end", "zz"])
def test_tiled_path_cnot_patterns(kind, tile_qubits):
    tile_qubits(6)
    c = cnot_pattern(10, kind)
    _run_expz_case(c, "c64", "hbm", 3, seed=4)


def test_tiled_path_c128(tile_qubits):
    tile_qubits(5)
    rng = np.random.default_rng(600)
    c = C.random_circuit(8, 60, rng, n_params=5, n_features=2)
    _run_expz_case(c, "c128", "hbm", 3, seed=3)


@pytest.mark.parametrize("n", [15, 16])
def test_large_state_auto_path(n):
    rng = np.random.default_rng(700 + n)
    c = C.random_circuit(n, 60, rng, n_params=6, n_features=1)
    assert N.qs_plan_info_get(N.CircuitHandle(c), N.QS_C64, 2)["path"] == N.QS_PATH_HBM
    _run_expz_case(c, "c64", "auto", 2, seed=n)


def test_c128_14_qubits_auto_path():
    rng = np.random.default_rng(714)
    c = C.random_circuit(14, 70, rng, n_params=6, n_features=2)
    assert N.qs_plan_info_get(N.CircuitHandle(c), N.QS_C128, 3)["path"] == N.QS_PATH_HBM
    _run_expz_case(c, "c128", "auto", 3, seed=14)
    _run_expz_case(c, "c128", "auto", 2, seed=15, per_sample=True)


def test_tiled_checkpoints(tile_qubits):
    tile_qubits(6)
    w = Dt.make_workload("c2", 3)
    c = w.circuit
    ck = c.layer_end[1:-1:3]
    s = sim.Simulator(c, "c64", PATHS["hbm"])
    st = s.encode_amplitude(_dev(w.x, torch.float32))
    buf = torch.empty((len(ck),) + tuple(st.shape), dtype=st.dtype, device="cuda")
    p = _dev(w.params, torch.float32)
    s.forward(p, None, st, ckpt_gates=ck, ckpt=buf)
    dz = torch.zeros(3, 10, dtype=torch.float64, device="cuda")
    dz[:, 0] = 0.2
    gp, _ = s.adjoint(p, None, st, dexpz=dz, ckpt_gates=ck, ckpt=buf)
    torch.cuda.synchronize()
    psi0 = O.encode_amplitude(w.x, 10)
    for i, g in enumerate(ck):
        ref = O.run_circuit(C.Circuit(10, c.gates[:g], c.n_params), w.params, None, psi0)
        np.testing.assert_allclose(buf[i].cpu().numpy(), ref, atol=1e-5)
    gth, _ = O.adjoint_vjp(c, w.params, None, psi0, dexpz=dz.cpu().numpy())
    np.testing.assert_allclose(gp.cpu().numpy(),
                               O.theta_to_param_grads(c, w.params, None, gth)[0], atol=1e-4)


def test_26q_structure_at_18_qubits_with_checkpoints_and_weighted_loss():
    """The 26-qubit workload's structure at a size the oracle carries: 18
    qubits (five outer bits around the default 13-qubit tile), 20
    hardware-efficient layers with ring CNOTs (CNOT folding across tile and
    outer bits), checkpoints every 4 layers, loss sum_q g_q <Z_q> with its
    gradient, one whole step on the automatic (tiled) path. Deep random
    circuits have small gradients, so the gradient is also held to a
    relative-norm bound."""
    n = 18
    _announce(f"26-qubit structure at n={n}, checkpoints every 4 layers")
    c = C.hea_ry_rz_ring(n, 20)
    w = Dt.Workload("hea ring n18 L20", n, 1, c, "c64", "zero", "weighted_z",
                    params=Dt.uniform_params(c.n_params, 0),
                    weights=Dt.upstream_weights(n, 0))
    d = sim.to_device(w, ckpt_every_layers=4)
    assert d.sim.plan_info(1)["path"] == N.QS_PATH_HBM
    assert d.ckpt_gates == [c.layer_end[l - 1] for l in (4, 8, 12, 16)]
    out = sim.step(d)
    torch.cuda.synchronize()
    p64 = w.params.astype(np.float64)
    psi0 = O.encode_zero(1, n)
    z = O.expz(O.run_circuit(c, p64, None, psi0))
    L, dz = O.loss_and_dexpz("weighted_z", z, None, w.weights)
    gth, _ = O.adjoint_vjp(c, p64, None, psi0, dexpz=dz)
    gp = O.theta_to_param_grads(c, p64, None, gth)[0]
    np.testing.assert_allclose(out["expz"].cpu().numpy(), z, atol=1e-5)
    assert abs(out["loss"].item() - L) < 1e-5 * n
    got = out["grad_params"].cpu().numpy()
    np.testing.assert_allclose(got, gp, atol=1e-4)
    assert np.linalg.norm(got - gp) <= 1e-3 * np.linalg.norm(gp)
    for i, g in enumerate(d.ckpt_gates):  # the stored states themselves
        ref = O.run_circuit(C.Circuit(n, c.gates[:g], c.n_params), p64, None, psi0)
        np.testing.assert_allclose(d.ckpt[i].cpu().numpy(), ref, atol=1e-5)


def test_tiled_checkpoints_that_widen_an_epochs_gradient_columns():
    """Shared-parameter circuits whose checkpoints give some epoch more
    gradient columns than any epoch of the plan without them: the workspace
    qs_workspace_size reports holds them, and the gradients match the oracle."""
    rng = np.random.default_rng(2024)
    found = 0
    for trial in range(200):
        n = int(rng.integers(15, 18))
        G = int(rng.integers(60, 240))
        P = int(rng.integers(2, 12))
        c = C.random_circuit(n, G, rng, n_params=P, n_features=0)
        B = int(rng.choice([1, 8, 32]))
        ck = sorted(set(int(v) for v in rng.integers(1, G, size=int(rng.integers(1, 5)))))
        if n > 16 or B < 8:
            continue
        h = N.CircuitHandle(c)
        a = N.qs_hbm_info_get(h, N.QS_C64, B, N.QS_PATH_HBM, ck)
        b = N.qs_hbm_info_get(h, N.QS_C64, B, N.QS_PATH_HBM)
        if a["max_partial_bytes"] <= b["max_partial_bytes"]:
            continue
        _announce(f"widened epoch: n={n} G={G} P={P} B={B} ckpt={ck}")
        s = sim.Simulator(c, "c64", PATHS["hbm"])
        x = rng.standard_normal((B, 1 << n)).astype(np.float32)
        st = s.encode_amplitude(_dev(x, torch.float32))
        buf = torch.empty((len(ck),) + tuple(st.shape), dtype=st.dtype, device="cuda")
        params = rng.uniform(-np.pi, np.pi, P).astype(np.float32)
        pt = _dev(params, torch.float32)
        s.forward(pt, None, st, ckpt_gates=ck, ckpt=buf)
        dz = rng.uniform(-1, 1, (B, n))
        ws = s.workspace(B)
        assert ws.numel() >= 2 * (B << n) * 8 + a["max_partial_bytes"]
        gp, _ = s.adjoint(pt, None, st, dexpz=_dev(dz, torch.float64), ws=ws,
                          ckpt_gates=ck, ckpt=buf)
        torch.cuda.synchronize()
        psi0 = O.encode_amplitude(x, n)
        gth, _ = O.adjoint_vjp(c, params, None, psi0, dexpz=dz)
        np.testing.assert_allclose(gp.cpu().numpy(),
                                   O.theta_to_param_grads(c, params, None, gth)[0],
                                   atol=1e-4)
        found += 1
        if found == 2:
            break
    assert found >= 1


# ------------------------------------- large states: dense blocks on MFMA
@pytest.mark.parametrize("n,G,B", [(10, 150, 3), (11, 90, 2), (13, 200, 2), (15, 120, 1)])
def test_mfma_block_path_random_circuits(n, G, B):
    """Every gate kind, shared parameters (including parameters read by
    several rotations and as biases), states, <Z> and gradients against the
    oracle; then a state cotangent."""
    rng = np.random.default_rng(1000 + n)
    c = C.random_circuit(n, G, rng, n_params=9, n_features=0)
    _run_expz_case(c, "c64", "mfma", B, seed=n)
    _run_expz_case(c, "c64", "mfma", B, seed=n + 1, dstate_mode=True, amplitude=False)


def test_mfma_block_path_checkpoints_and_inverse():
    rng = np.random.default_rng(1017)
    n, G, B = 12, 160, 2
    c = C.random_circuit(n, G, rng, n_params=8, n_features=0)
    ck = [17, 60, 61, 140]
    s = sim.Simulator(c, "c64", PATHS["mfma"])
    x = rng.standard_normal((B, 1 << n)).astype(np.float32)
    st = s.encode_amplitude(_dev(x, torch.float32))
    buf = torch.empty((len(ck),) + tuple(st.shape), dtype=st.dtype, device="cuda")
    params = rng.uniform(-np.pi, np.pi, c.n_params).astype(np.float32)
    pt = _dev(params, torch.float32)
    z = s.forward(pt, None, st, ckpt_gates=ck, ckpt=buf)
    dz = rng.uniform(-1, 1, (B, n))
    gp, _ = s.adjoint(pt, None, st, dexpz=_dev(dz, torch.float64), ckpt_gates=ck, ckpt=buf)
    torch.cuda.synchronize()
    psi0 = O.encode_amplitude(x, n)
    for i, g in enumerate(ck):
        ref = O.run_circuit(C.Circuit(n, c.gates[:g], c.n_params), params, None, psi0)
        np.testing.assert_allclose(buf[i].cpu().numpy(), ref, atol=1e-5)
    np.testing.assert_allclose(z.cpu().numpy(), O.expz(O.run_circuit(c, params, None, psi0)),
                               atol=1e-5)
    gth, _ = O.adjoint_vjp(c, params, None, psi0, dexpz=dz)
    np.testing.assert_allclose(gp.cpu().numpy(),
                               O.theta_to_param_grads(c, params, None, gth)[0], atol=1e-4)
    # the inverse flag runs U^dagger: back to the input
    s.forward(pt, None, st, want_expz=False, flags=PATHS["mfma"] | N.QS_FLAG_INVERSE)
    torch.cuda.synchronize()
    np.testing.assert_allclose(st.cpu().numpy(), psi0, atol=1e-5)


def test_26q_structure_at_18_qubits_on_mfma_blocks():
    """The 18-qubit version of the 26-qubit workload (see the tiled-path test
    above) on the dense-block MFMA path."""
    n = 18
    _announce(f"26-qubit structure at n={n} on MFMA blocks")
    c = C.hea_ry_rz_ring(n, 20)
    w = Dt.Workload("hea ring n18 L20", n, 1, c, "c64", "zero", "weighted_z",
                    params=Dt.uniform_params(c.n_params, 0),
                    weights=Dt.upstream_weights(n, 0))
    d = sim.to_device(w, flags=PATHS["mfma"], ckpt_every_layers=4)
    out = sim.step(d)
    torch.cuda.synchronize()
    p64 = w.params.astype(np.float64)
    psi0 = O.encode_zero(1, n)
    z = O.expz(O.run_circuit(c, p64, None, psi0))
    L, dz = O.loss_and_dexpz("weighted_z", z, None, w.weights)
    gth, _ = O.adjoint_vjp(c, p64, None, psi0, dexpz=dz)
    gp = O.theta_to_param_grads(c, p64, None, gth)[0]
    np.testing.assert_allclose(out["expz"].cpu().numpy(), z, atol=1e-5)
    got = out["grad_params"].cpu().numpy()
    np.testing.assert_allclose(got, gp, atol=1e-4)
    assert np.linalg.norm(got - gp) <= 1e-3 * np.linalg.norm(gp)


def test_full_size_26q_on_mfma_blocks_closed_forms_and_inverse():
    """26 qubits on the MFMA path: the product circuit's per-qubit closed
    forms and gradients, and the hardware-efficient circuit then its inverse
    returning |0...0>."""
    _announce("26-qubit product state on MFMA blocks")
    n = 26
    rng = np.random.default_rng(826)
    c = _product_circuit(n, 3, rng)
    params = rng.uniform(-np.pi, np.pi, c.n_params).astype(np.float32)
    g = rng.uniform(-1, 1, n)
    s = sim.Simulator(c, "c64", PATHS["mfma"])
    st = s.zero_state(1)
    pt = _dev(params, torch.float32)
    z = s.forward(pt, None, st)
    gp, _ = s.adjoint(pt, None, st, dexpz=_dev(g[None, :], torch.float64))
    torch.cuda.synchronize()
    z = z.cpu().numpy()[0]
    gp = gp.cpu().numpy()
    for q in range(n):
        sel = [i for i, gt in enumerate(c.gates) if gt["q0"] == q]
        g1 = c.gates[sel].copy()
        g1["q0"] = 0
        c1 = C.Circuit(1, g1, c.n_params)
        psi = O.run_circuit(c1, params, None, O.encode_zero(1, 1))
        assert abs(z[q] - O.expz(psi)[0, 0]) < 1e-5
        gth, _ = O.adjoint_vjp(c1, params, None, O.encode_zero(1, 1),
                               dexpz=np.array([[g[q]]]))
        ref = O.theta_to_param_grads(c1, params, None, gth)[0]
        idx = np.unique(g1["p_w"])
        np.testing.assert_allclose(gp[idx], ref[idx], atol=1e-4)
    del st
    _announce("26-qubit U then U^dagger on MFMA blocks")
    w = Dt.make_workload("c5b")
    s = sim.Simulator(w.circuit, "c64", PATHS["mfma"])
    st = s.zero_state(1)
    pt = _dev(w.params, torch.float32)
    s.forward(pt, None, st, want_expz=False)
    s.forward(pt, None, st, want_expz=False, flags=PATHS["mfma"] | N.QS_FLAG_INVERSE)
    torch.cuda.synchronize()
    assert abs(st[0, 0].item() - 1.0) < 1e-3
    norm = float((st.abs().double() ** 2).sum().item())
    assert abs(norm - 1.0) < 1e-3


def _product_circuit(n, layers, rng):
    """RY then RZ on every qubit, `layers` times, no entanglers: each qubit
    evolves alone, so the oracle can check <Z_q> and its gradient qubit by
    qubit at any n."""
    b = C._Builder(n)
    for _ in range(layers):
        for q in range(n):
            b.rot("RY", q, p_w=b.new_param())
            b.rot("RZ", q, p_w=b.new_param())
            b.rot("RX", q, p_w=b.new_param())
    return b.build()


@pytest.mark.parametrize("n", [20, 26])
def test_full_size_product_state_closed_forms(n):
    """Full-size large states on the tiled path: per-qubit closed forms for
    <Z_q> and for dL/dP of L = sum_q g_q <Z_q>, computed by the oracle on each
    qubit's own 1-qubit circuit."""
    _announce(f"product state n={n}")
    rng = np.random.default_rng(800 + n)
    c = _product_circuit(n, 3, rng)
    P = c.n_params
    params = rng.uniform(-np.pi, np.pi, P).astype(np.float32)
    g = rng.uniform(-1, 1, n)
    s = sim.Simulator(c, "c64")
    st = s.zero_state(1)
    pt = _dev(params, torch.float32)
    z = s.forward(pt, None, st)
    gp, _ = s.adjoint(pt, None, st, dexpz=_dev(g[None, :], torch.float64))
    torch.cuda.synchronize()
    norm = float((st.abs().double() ** 2).sum().item())
    assert abs(norm - 1.0) < 1e-5
    z = z.cpu().numpy()[0]
    gp = gp.cpu().numpy()
    for q in range(n):
        sel = [i for i, gt in enumerate(c.gates) if gt["q0"] == q]
        g1 = c.gates[sel].copy()
        g1["q0"] = 0
        c1 = C.Circuit(1, g1, P)
        psi = O.run_circuit(c1, params, None, O.encode_zero(1, 1))
        assert abs(z[q] - O.expz(psi)[0, 0]) < 1e-5
        gth, _ = O.adjoint_vjp(c1, params, None, O.encode_zero(1, 1),
                               dexpz=np.array([[g[q]]]))
        ref = O.theta_to_param_grads(c1, params, None, gth)[0]
        idx = np.unique(g1["p_w"])
        np.testing.assert_allclose(gp[idx], ref[idx], atol=1e-4)


def test_full_size_26q_circuit_then_inverse_is_identity():
    """The 26-qubit hardware-efficient circuit (20 layers, 1560 gates) followed
    by its inverse returns |0...0> exactly (up to rounding), and the forward
    alone preserves the norm."""
    w = Dt.make_workload("c5b")
    _announce("26-qubit U then U^dagger")
    c = w.circuit
    inv = C.inverse_structure(c)
    s = sim.Simulator(c, "c64")
    si = sim.Simulator(inv, "c64")
    st = s.zero_state(1)
    pt = _dev(w.params, torch.float32)
    z = s.forward(pt, None, st)
    torch.cuda.synchronize()
    # In complex64 each rotation's cos and sin are rounded to float, so
    # c^2 + s^2 = 1 + d with |d| <= 2 * 2^-23 (two roundings of 2^-24 each,
    # doubled by squaring), and every rotation scales the whole norm by that
    # factor. The drift is therefore bounded by n_rot * 2^-22 (systematic,
    # growing linearly with depth); the random per-amplitude rounding adds only
    # about sqrt(G) * 6e-8 on top.
    n_rot = int(np.isin(c.gates["op"], list(C.ROTATIONS)).sum())
    tol = n_rot * 2.0 ** -22
    norm = float((st.abs().double() ** 2).sum().item())
    assert abs(norm - 1.0) < tol, (norm, tol)
    assert np.all(np.abs(z.cpu().numpy()) <= 1 + tol)
    si.forward(pt, None, st, want_expz=False)
    torch.cuda.synchronize()
    a0 = st[0, 0].item()
    # U^dagger repeats the norm drift with the same bound.
    assert abs(a0 - 1.0) < 2 * tol + 1e-5, (a0, tol)


# ------------------------------------------------------- uneven batches
def _oracle_program_circuit(ub, k, j):
    n, d, c, idx = ub.classes[k]
    xs, ps, es = ub.circuit_slices(k, j)
    x = ub.x[xs][None, :]
    p = ub.params[ps]
    g = ub.weights[es][None, :]
    psi0 = O.encode_amplitude(x, n)
    z = O.expz(O.run_circuit(c, p, None, psi0))
    gth, _ = O.adjoint_vjp(c, p, None, psi0, dexpz=g)
    return z[0], O.theta_to_param_grads(c, p, None, gth)[0]


def test_uneven_batch_small_all_circuits():
    ub = Dt.uneven_batch(90, seed=3, n_lo=5, n_hi=10, d_lo=1, d_hi=4)
    _announce(f"uneven batch: {ub.n_circuits} circuits, {len(ub.classes)} classes")
    dev = sim.UnevenDevice(ub)
    out = dev.step()
    torch.cuda.synchronize()
    z = out["expz"].cpu().numpy()
    gp = out["grad_params"].cpu().numpy()
    for k, (n, d, c, idx) in enumerate(ub.classes):
        for j in range(len(idx)):
            zo, go = _oracle_program_circuit(ub, k, j)
            _, ps, es = ub.circuit_slices(k, j)
            np.testing.assert_allclose(z[es], zo, atol=1e-5)
            np.testing.assert_allclose(gp[ps], go, atol=1e-4)


def test_uneven_batch_table_and_on_the_fly_classes():
    """Deep 11- and 12-qubit classes: the persistent kernel keeps an LDS
    angle table for the classes where it fits beside the staging (12 qubits:
    4 circuits per workgroup) and computes angles in place for the others
    (11 qubits at depth 32: 8 circuits x 704 angles do not fit); every
    circuit of both kinds matches the oracle."""
    ub = Dt.uneven_batch(10, seed=13, n_lo=11, n_hi=12, d_lo=20, d_hi=32)
    assert any(n == 11 and d > 24 for n, d, _, _ in ub.classes)
    _announce(f"uneven batch table/fly: {ub.n_circuits} circuits, {len(ub.classes)} classes")
    dev = sim.UnevenDevice(ub)
    out = dev.step()
    torch.cuda.synchronize()
    z = out["expz"].cpu().numpy()
    gp = out["grad_params"].cpu().numpy()
    for k, (n, d, c, idx) in enumerate(ub.classes):
        for j in range(len(idx)):
            zo, go = _oracle_program_circuit(ub, k, j)
            _, ps, es = ub.circuit_slices(k, j)
            np.testing.assert_allclose(z[es], zo, atol=1e-5)
            np.testing.assert_allclose(gp[ps], go, atol=1e-4)


def test_uneven_batch_c128():
    ub = Dt.uneven_batch(40, seed=5, n_lo=4, n_hi=9, d_lo=1, d_hi=3)
    _announce(f"uneven batch c128: {ub.n_circuits} circuits, {len(ub.classes)} classes")
    dev = sim.UnevenDevice(ub, dtype="c128")
    out = dev.step()
    torch.cuda.synchronize()
    z = out["expz"].cpu().numpy()
    gp = out["grad_params"].cpu().numpy()
    for k, (n, d, c, idx) in enumerate(ub.classes):
        for j in range(len(idx)):
            zo, go = _oracle_program_circuit(ub, k, j)
            _, ps, es = ub.circuit_slices(k, j)
            np.testing.assert_allclose(z[es], zo, atol=1e-10)
            np.testing.assert_allclose(gp[ps], go, atol=1e-10)


def test_uneven_batch_c128_wide():
    """Classes up to 14 qubits in complex128: the program stages one state
    component at a time in LDS when whole amplitudes do not fit."""
    ub = Dt.uneven_batch(24, seed=7, n_lo=12, n_hi=14, d_lo=2, d_hi=6)
    _announce(f"uneven batch c128 wide: {ub.n_circuits} circuits, {len(ub.classes)} classes")
    dev = sim.UnevenDevice(ub, dtype="c128")
    out = dev.step()
    torch.cuda.synchronize()
    z = out["expz"].cpu().numpy()
    gp = out["grad_params"].cpu().numpy()
    for k, (n, d, c, idx) in enumerate(ub.classes):
        for j in range(len(idx)):
            zo, go = _oracle_program_circuit(ub, k, j)
            _, ps, es = ub.circuit_slices(k, j)
            np.testing.assert_allclose(z[es], zo, atol=1e-10)
            np.testing.assert_allclose(gp[ps], go, atol=1e-10)


def test_uneven_batch_full_size_sampled():
    ub = Dt.uneven_batch()
    _announce(f"uneven batch full: {ub.n_circuits} circuits, {len(ub.classes)} classes")
    dev = sim.UnevenDevice(ub)
    out = dev.step()
    torch.cuda.synchronize()
    z = out["expz"].cpu().numpy()
    gp = out["grad_params"].cpu().numpy()
    assert np.all(np.abs(z) <= 1 + 1e-5)
    rng = np.random.default_rng(11)
    picks = [(0, 0), (len(ub.classes) - 1, 0)] + \
        [(int(k), 0) for k in rng.integers(0, len(ub.classes), 4)]
    for k, j in picks:
        zo, go = _oracle_program_circuit(ub, k, j)
        _, ps, es = ub.circuit_slices(k, j)
        np.testing.assert_allclose(z[es], zo, atol=1e-5)
        g = gp[ps]
        assert np.abs(g - go).max() < 1e-4 or \
            np.linalg.norm(g - go) <= 1e-3 * np.linalg.norm(go)


def test_graph_replay_matches_eager():
    """A captured step replayed several times, with eager work in between,
    reproduces the eager result every time (the batched and the uneven path)."""
    w = Dt.make_workload("c2", 64)
    d = sim.to_device(w)
    eager = sim.step(d)
    ref_z = eager["expz"].clone()
    ref_g = eager["grad_params"].clone()
    gs = sim.GraphStep(lambda: sim.step(d))
    for rep in range(3):
        out = gs.replay()
        torch.cuda.synchronize()
        assert torch.equal(out["expz"], ref_z), rep
        assert torch.allclose(out["grad_params"], ref_g, rtol=0, atol=1e-12), rep
        sim.step(d)  # eager work between replays
        torch.cuda.synchronize()
    ub = Dt.uneven_batch(60, seed=5, n_lo=5, n_hi=9, d_lo=1, d_hi=3)
    dev = sim.UnevenDevice(ub)
    e = dev.step()
    rz, rg = e["expz"].clone(), e["grad_params"].clone()
    gu = sim.GraphStep(lambda: dev.step())
    for rep in range(3):
        out = gu.replay()
        torch.cuda.synchronize()
        assert torch.equal(out["expz"], rz), rep
        assert torch.allclose(out["grad_params"], rg, rtol=0, atol=1e-12), rep
        dev.step()
        torch.cuda.synchronize()


def test_graph_replay_uneven_with_side_streams():
    """Complex128 classes of 14 qubits run on the program's side streams; a
    captured step (fork and join inside the graph) replays to the eager
    result, with eager work between the replays."""
    ub = Dt.uneven_batch(16, seed=9, n_lo=13, n_hi=14, d_lo=1, d_hi=3)
    assert any(n == 14 for n, _, _, _ in ub.classes)
    _announce(f"graph replay, uneven c128 with side streams: {len(ub.classes)} classes")
    dev = sim.UnevenDevice(ub, dtype="c128")
    e = dev.step()
    torch.cuda.synchronize()
    rz, rg = e["expz"].clone(), e["grad_params"].clone()
    gu = sim.GraphStep(lambda: dev.step())
    for rep in range(3):
        out = gu.replay()
        torch.cuda.synchronize()
        assert torch.allclose(out["expz"], rz, rtol=0, atol=1e-12), rep
        assert torch.allclose(out["grad_params"], rg, rtol=0, atol=1e-12), rep
        dev.step()
        torch.cuda.synchronize()


def test_shutdown_then_replan_gives_the_same_results():
    """qs_shutdown releases every cached plan, program plans (which point into
    the engine plans) included; the next calls plan again and agree with the
    first (batched, uneven, and uneven with side streams)."""
    torch.cuda.synchronize()
    w = Dt.make_workload("c2", 32)
    d = sim.to_device(w)
    a = sim.step(d)
    ub = Dt.uneven_batch(12, seed=4, n_lo=12, n_hi=14, d_lo=1, d_hi=2)
    dev = sim.UnevenDevice(ub, dtype="c128")
    u = dev.step()
    torch.cuda.synchronize()
    ref = [a["expz"].clone(), a["grad_params"].clone(), u["expz"].clone(),
           u["grad_params"].clone()]
    N.qs_shutdown()
    a = sim.step(d)
    u = dev.step()
    torch.cuda.synchronize()
    for x, y in zip(ref, [a["expz"], a["grad_params"], u["expz"], u["grad_params"]]):
        assert torch.allclose(x, y, rtol=0, atol=1e-12)


# ------------------------------------------------------------- autotuner
def test_autotune_picks_a_config_and_results_stay_exact(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("QS_AUTOTUNE_CACHE", str(cache))
    w = Dt.make_workload("c2", 96)
    s = sim.Simulator(w.circuit, "c64")
    info = N.qs_autotune(s.h, s.qs_dtype, 96)
    torch.cuda.synchronize()
    assert info["path"] == N.QS_PATH_FUSED
    assert info["fwd_log2_regs"] in (1, 2, 3, 4, 5) and info["adj_log2_regs"] in (1, 2, 3, 4, 5)
    assert info["n_candidates"] >= 2 and info["fwd_ms"] > 0 and info["adj_ms"] > 0
    line = cache.read_text().split()
    assert int(line[1]) == info["fwd_log2_regs"] and int(line[2]) == info["adj_log2_regs"]
    assert int(line[4]) == info["fwd_samples_cap"] and int(line[5]) == info["adj_samples_cap"]
    assert int(line[6]) == info["fwd_half_staging"] and int(line[7]) == info["adj_half_staging"]
    pi = s.plan_info(96)
    assert pi["log2_regs"] == info["fwd_log2_regs"]
    assert pi["adj_log2_regs"] == info["adj_log2_regs"]
    for cap, S, r in ((info["fwd_samples_cap"], pi["samples_per_block"], pi["log2_regs"]),
                      (info["adj_samples_cap"], pi["adj_samples_per_block"],
                       pi["adj_log2_regs"])):
        whole_wave = max(1, 64 >> (10 - r))  # a block keeps whole waves
        assert cap == 0 or S <= max(cap, whole_wave)
    test_workload_step_vs_oracle("c2", 96)  # the tuned configuration is exact too
