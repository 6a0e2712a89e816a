"""Host-side tests of libqs.so that need no GPU: the library loads, exports
every call include/qs.h declares, its descriptor constants match the
workload generator's, descriptor validation rejects malformed input, and the
planner's programs respect the circuit (same per-qubit gate order, every
pair-mixing gate on a register-resident qubit)."""
import os
import ctypes
import re

import numpy as np
import pytest

from paper_2509_25075_amd import _native as N
from workloads import circuits as C
from workloads import data as Dt
from _patterns import cnot_pattern

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "qs.h")


def _header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(qs_\w+)\s*\(", txt, flags=re.M)))


def test_library_loads_and_exports_every_declared_call():
    lib = N.lib()
    names = _header_functions()
    assert len(names) >= 12, names
    for name in names:
        assert hasattr(lib, name), f"libqs.so does not export {name}"
    assert N.qs_version() == 10000


def test_header_constants_match_descriptor_format():
    txt = open(HEADER).read()
    for name, val in C.OP.items():
        m = re.search(rf"QS_OP_{name}\s*=\s*(\d+)", txt)
        assert m and int(m.group(1)) == val, name
    for const in ["QS_C64", "QS_C128", "QS_ENC_AMPLITUDE", "QS_ENC_ZERO",
                  "QS_PATH_AUTO", "QS_PATH_FUSED", "QS_PATH_PLAIN", "QS_PATH_HBM"]:
        m = re.search(rf"\b{const}\s*=\s*(\d+)", txt)
        assert m and int(m.group(1)) == getattr(N, const), const
    m = re.search(r"QS_FLAG_PER_SAMPLE_PARAMS\s*=\s*(0x[0-9a-f]+)", txt)
    assert int(m.group(1), 16) == N.QS_FLAG_PER_SAMPLE_PARAMS
    assert C.GATE_DTYPE == N.GATE_NP_DTYPE
    assert C.GATE_DTYPE.itemsize == 32


def test_fidelity_calls_validate_before_touching_the_gpu():
    """Bad sizes are rejected and B = 0 is a no-op, before any device work
    (so these run without a GPU)."""
    L = N.lib()
    nul = [None] * 7
    # n_trash must be < n (and <= 6 where the kernel keeps per-outcome sums)
    assert L.qs_fidelity_postselect(N.QS_C64, 4, 4, 1, *nul) == N.QS_ERR_INVALID
    assert L.qs_fidelity_trajectory(N.QS_C64, 10, 7, 1, *nul, None, None) == N.QS_ERR_INVALID
    assert L.qs_fidelity_reset(N.QS_C64, 10, 7, 1, *nul) == N.QS_ERR_INVALID
    assert L.qs_fidelity_postselect(3, 4, 1, 1, *nul) == N.QS_ERR_INVALID     # dtype
    assert L.qs_fidelity_trajectory(N.QS_C128, 31, 1, 1, *nul, None, None) == N.QS_ERR_INVALID
    # missing buffers with B > 0
    assert L.qs_fidelity_postselect(N.QS_C64, 4, 1, 2, *nul) == N.QS_ERR_INVALID
    assert L.qs_fidelity_trajectory(N.QS_C64, 4, 1, 2, *nul, None, None) == N.QS_ERR_INVALID
    # B = 0: nothing to do, no buffers needed
    assert L.qs_fidelity_reset(N.QS_C64, 4, 1, 2, *nul) == N.QS_ERR_INVALID
    assert L.qs_fidelity_reset(N.QS_C64, 4, 1, 1 << 31, *nul) == N.QS_ERR_INVALID  # B bound
    assert L.qs_fidelity_postselect(N.QS_C64, 4, 1, 1 << 31, *nul) == N.QS_ERR_INVALID
    # B = 0: nothing to do, no buffers needed
    assert L.qs_fidelity_postselect(N.QS_C64, 4, 1, 0, *nul) == N.QS_OK
    assert L.qs_fidelity_trajectory(N.QS_C128, 4, 2, 0, *nul, None, None) == N.QS_OK
    assert L.qs_fidelity_reset(N.QS_C64, 4, 1, 0, *nul) == N.QS_OK


def test_forward_amplitude_and_loss_validate_before_touching_the_gpu():
    """Bad encoding arguments and bad loss shapes are rejected, and B = 0 is a
    no-op, before any device work."""
    L = N.lib()
    h = N.CircuitHandle(C.hea_ry_rz_ring(3, 1))
    x = ctypes.c_void_p(16)  # never dereferenced: every call below returns first
    args = lambda B, xp, D, xs: (h.ptr, N.QS_C64, B, x, None, xp, 0, D, xs, None, x,
                                 None, None, 0, None, 0, None)
    assert L.qs_forward_amplitude(*args(2, None, 8, 8)) == N.QS_ERR_INVALID   # no x
    assert L.qs_forward_amplitude(*args(2, x, 0, 8)) == N.QS_ERR_INVALID      # D < 1
    assert L.qs_forward_amplitude(*args(2, x, 9, 9)) == N.QS_ERR_INVALID      # D > 2^n
    assert L.qs_forward_amplitude(*args(2, x, 8, 7)) == N.QS_ERR_INVALID      # stride < D
    assert L.qs_forward_amplitude(*args(0, None, 0, 0)) == N.QS_OK            # B = 0
    assert L.qs_loss_mse_z(0, 4, 0, x, x, x, x, None) == N.QS_ERR_INVALID     # n < 1
    assert L.qs_loss_mse_z(3, 4, 3, x, x, x, x, None) == N.QS_ERR_INVALID     # q >= n
    assert L.qs_loss_mse_z(3, 4, -1, x, x, x, x, None) == N.QS_ERR_INVALID
    assert L.qs_loss_mse_z(3, -1, 0, x, x, x, x, None) == N.QS_ERR_INVALID    # B < 0
    assert L.qs_loss_mse_z(3, 4, 0, None, x, x, x, None) == N.QS_ERR_INVALID  # no expz
    assert L.qs_loss_mse_z(3, 4, 0, x, None, x, x, None) == N.QS_ERR_INVALID  # no y
    assert L.qs_loss_mse_z(3, 4, 0, x, x, None, None, None) == N.QS_OK        # no outputs


def test_train_step_validates_before_touching_the_gpu():
    """The one-launch training step rejects bad arguments and shapes it has
    no kernel for before any device work; its workspace query is host-only."""
    L = N.lib()
    c = C.hea_ry_rz_ring(3, 1)
    h = N.CircuitHandle(c)
    p = ctypes.c_void_p(16)  # never dereferenced: every call below returns first

    def call(B=4, q=0, dtype=N.QS_C64, x=None, f64=0, y=p, loss=p, flags=0):
        return L.qs_train_step_mse(h.ptr, dtype, B, p, None, x, f64, 8, 8, None, y, q, None,
                                   loss, p, None, p, 1 << 20, flags, None)
    assert call(q=3) == N.QS_ERR_INVALID          # q >= n
    assert call(q=-1) == N.QS_ERR_INVALID
    assert call(B=-1) == N.QS_ERR_INVALID
    assert call(y=None) == N.QS_ERR_INVALID
    assert call(loss=None) == N.QS_ERR_INVALID
    assert call(B=0, y=None, loss=None) == N.QS_OK  # nothing to do
    assert call(x=p, f64=1) == N.QS_ERR_UNSUPPORTED  # complex64 reads float32 inputs
    assert call(dtype=N.QS_C128) == N.QS_ERR_UNSUPPORTED
    assert call(flags=N.QS_FLAG_PER_SAMPLE_PARAMS) == N.QS_ERR_UNSUPPORTED
    # workspace query: > 0 where the kernel runs, 0 otherwise
    w2 = Dt.make_workload("c2", 4096)
    h2 = N.CircuitHandle(w2.circuit)
    assert N.qs_train_workspace_size(h2, N.QS_C64, 4096) > 0
    assert N.qs_train_workspace_size(h2, N.QS_C128, 4096) == 0
    assert N.qs_train_workspace_size(h2, N.QS_C64, 4096, N.QS_FLAG_PER_SAMPLE_PARAMS) == 0
    assert N.qs_train_workspace_size(h2, N.QS_C64, 0) == 0


def test_status_strings():
    for s in [0, -1, -2, -3, -4, -5, -6, -7, -8, 7]:
        assert isinstance(N.status_string(s), str) and N.status_string(s)
    assert "capture" in N.status_string(N.QS_ERR_CAPTURE)
    assert N.status_string(-7) != N.status_string(7)
    txt = open(HEADER).read()
    assert int(re.search(r"QS_ERR_CAPTURE\s*=\s*(-\d+)", txt).group(1)) == N.QS_ERR_CAPTURE
    assert N.lib().qs_encode_check(None, None) == N.QS_ERR_INVALID


def _circ(n, rows, n_params=4, n_features=2):
    return C.Circuit(n, np.array(rows, dtype=C.GATE_DTYPE), n_params, n_features)


@pytest.mark.parametrize("rows,n,why", [
    ([(0, 3, -1, 0, -1, -1, 1.0, 0)], 3, "qubit out of range"),
    ([(0, -1, -1, 0, -1, -1, 1.0, 0)], 3, "negative qubit"),
    ([(99, 0, -1, -1, -1, -1, 1.0, 0)], 3, "unknown op"),
    ([(7, 1, 1, -1, -1, -1, 0.0, 0)], 3, "CNOT control = target"),
    ([(8, 0, 5, -1, -1, -1, 0.0, 0)], 3, "CZ second qubit out of range"),
    ([(0, 0, 1, 0, -1, -1, 1.0, 0)], 3, "1-qubit gate with q1"),
    ([(1, 0, -1, 4, -1, -1, 1.0, 0)], 3, "weight index >= n_params"),
    ([(1, 0, -1, -1, -1, 7, 1.0, 0)], 3, "bias index >= n_params"),
    ([(2, 0, -1, -1, 2, -1, 1.0, 0)], 3, "feature index >= n_features"),
    ([(2, 0, -1, -1, -1, -1, 1.0, 1)], 3, "nonzero flags"),
    ([], 0, "zero qubits"),
    ([], 31, "too many qubits"),
])
def test_validate_rejects(rows, n, why):
    h = N.CircuitHandle(_circ(n, rows))
    assert N.qs_validate(h) == N.QS_ERR_INVALID, why


def test_validate_accepts_workloads_and_random():
    for key in ["c1", "c2", "c3", "c4"]:
        w = Dt.make_workload(key, 2)
        assert N.qs_validate(N.CircuitHandle(w.circuit)) == N.QS_OK
    rng = np.random.default_rng(0)
    for n in range(1, 9):
        c = C.random_circuit(n, 50, rng, n_params=5, n_features=3)
        assert N.qs_validate(N.CircuitHandle(c)) == N.QS_OK
    assert N.qs_validate(N.CircuitHandle(_circ(3, []))) == N.QS_OK


MIXING = {C.OP[k] for k in ("RX", "RY", "X", "Y", "H")}


def _check_plan(c, dtype, flags=0, B=8):
    h = N.CircuitHandle(c)
    info, ops, sb, sm = N.qs_plan_export(h, dtype, B, flags)
    r = info["log2_regs"]
    n = c.n_qubits
    assert info["log2_regs"] + info["log2_threads"] == n
    G = c.n_gates
    # every gate exactly once
    assert sorted(ops[:, 3].tolist()) == list(range(G))
    # per-qubit order kept: any topological order of the dependency DAG
    for q in range(n):
        touch = [g for g in ops[:, 3] if c.gates[g]["q0"] == q or c.gates[g]["q1"] == q]
        assert touch == sorted(touch)
    assert sb[0] == 0 and sb[-1] == G and np.all(np.diff(sb) >= 0)
    remaps = 0
    for s in range(info["n_segments"]):
        m = sm[s, :n]
        assert sorted(m.tolist()) == list(range(n)), "placement is a permutation"
        # a remap follows unless the previous segment's end layout (its
        # placement mapped through the CNOTs folded at its end) is this
        # segment's placement
        if s:
            lay = [1 << int(q) for q in sm[s - 1, :n]]
            for o in range(sb[s - 1], sb[s]):
                if ops[o, 1] < 0:
                    gc, gt = c.gates[ops[o, 3]]["q0"], c.gates[ops[o, 3]]["q1"]
                    lay = [v ^ (((v >> gc) & 1) << gt) for v in lay]
            if lay != [1 << int(q) for q in m]:
                remaps += 1
        for o in range(sb[s], sb[s + 1]):
            kind, a, b, g = ops[o]
            gate = c.gates[g]
            assert kind == gate["op"]
            if a < 0:
                # a CNOT folded into the remap that closes this segment
                assert kind == C.OP["CNOT"] and b < 0
                continue
            assert m[a] == gate["q0"]
            if gate["q1"] >= 0:
                assert m[b] == gate["q1"]
            if kind in MIXING:
                assert a < r, "pair-mixing target on a register bit"
            assert kind != C.OP["CNOT"], "CNOTs are folded into remaps"
    assert remaps == info["n_remaps"]
    return info


@pytest.mark.parametrize("key", ["c1", "c2", "c3", "c4"])
def test_plans_of_workloads(key):
    w = Dt.make_workload(key, 8)
    dt = N.QS_C128 if w.dtype == "c128" else N.QS_C64
    info = _check_plan(w.circuit, dt)
    assert info["path"] == N.QS_PATH_FUSED
    assert info["n_engine_ops"] <= info["n_ops"]
    if key == "c2":
        # one re-placement per layer: 8 layers of 10-qubit rotations, 5
        # register qubits, commuting gates reordered across the CZ ring
        assert info["n_remaps"] == 8
        # layer ops: per layer the 30 rotations become two fused-block ops
        # (5 register bits each) and the 10 CZs at most two sign-pattern ops
        assert info["n_engine_ops"] <= 4 * 8


@pytest.mark.parametrize("n", list(range(1, 15)))
def test_plans_of_random_circuits(n):
    rng = np.random.default_rng(n)
    c = C.random_circuit(n, 120, rng, n_params=6, n_features=2)
    for dt in (N.QS_C64, N.QS_C128):
        if dt == N.QS_C128 and n > 13:
            continue
        _check_plan(c, dt)
        _check_plan(c, dt, flags=N.QS_FLAG_PER_SAMPLE_PARAMS)


@pytest.mark.parametrize("kind", ["start_end", "zz", "cancel", "only"])
@pytest.mark.parametrize("n", [3, 7, 11])
def test_plans_fold_cnots_into_remaps(n, kind):
    c = cnot_pattern(n, kind)
    info = _check_plan(c, N.QS_C64)
    _check_plan(c, N.QS_C64, flags=N.QS_FLAG_PER_SAMPLE_PARAMS)
    if kind == "only":
        # chain, ring and chain again: one remap carries all of them
        assert info["n_engine_ops"] == 0 and info["n_remaps"] == 1


def test_large_circuits_take_the_tiled_path():
    c = C.hea_ry_rz_ring(16, 1)
    info = N.qs_plan_info_get(N.CircuitHandle(c), N.QS_C64, 1)
    assert info["path"] == N.QS_PATH_HBM
    assert info["log2_threads"] == 13 and info["n_segments"] >= 2  # tile qubits, epochs
    w = Dt.make_workload("c5b")
    info = N.qs_plan_info_get(N.CircuitHandle(w.circuit), N.QS_C64, 1)
    assert info["path"] == N.QS_PATH_HBM
    # 20 hardware-efficient layers on 26 qubits in 13-qubit tiles
    assert 40 <= info["n_segments"] <= 80
    plain = N.qs_plan_info_get(N.CircuitHandle(c), N.QS_C64, 1, N.QS_PATH_PLAIN)
    assert plain["path"] == N.QS_PATH_PLAIN
    # complex128 at 14 qubits does not fit one workgroup's registers and LDS:
    # the automatic path gathers 12-qubit tiles rather than going gate by gate
    h14 = N.CircuitHandle(C.hea_ry_rz_ring(14, 2))
    assert N.qs_plan_info_get(h14, N.QS_C64, 4)["path"] == N.QS_PATH_FUSED
    info = N.qs_plan_info_get(h14, N.QS_C128, 4)
    assert info["path"] == N.QS_PATH_HBM and info["log2_threads"] == 12


@pytest.mark.parametrize("dtype", [N.QS_C64, N.QS_C128])
def test_tiled_workspace_covers_checkpointed_plans(dtype):
    """Checkpoints move the large-state path's epoch boundaries, so an epoch
    can read more shared-parameter gradient columns than any epoch of the
    plan without them; the workspace qs_workspace_size reports (the same for
    every checkpoint set) must hold the partial sums of every epoch of every
    such plan."""
    rng = np.random.default_rng(2024)
    checked = grew = 0
    for trial in range(60):
        n = int(rng.integers(15, 18))
        G = int(rng.integers(60, 240))
        P = int(rng.integers(2, 12))  # few parameters, shared by many rotations
        c = C.random_circuit(n, G, rng, n_params=P, n_features=0)
        h = N.CircuitHandle(c)
        B = int(rng.choice([1, 8, 32]))
        k = int(rng.integers(1, 5))
        ck = sorted(set(int(v) for v in rng.integers(1, G, size=k)))
        try:
            info = N.qs_hbm_info_get(h, dtype, B, N.QS_PATH_HBM, ck)
        except N.QsError as e:
            assert e.status == N.QS_ERR_UNSUPPORTED
            continue
        base = N.qs_hbm_info_get(h, dtype, B, N.QS_PATH_HBM)
        ws = N.qs_workspace_size(h, dtype, B, N.QS_PATH_HBM)
        assert ws == info["ws_bytes"] == base["ws_bytes"]
        states = 2 * (B << n) * (8 if dtype == N.QS_C64 else 16)
        assert ws >= states + info["max_partial_bytes"], (trial, ck)
        assert ws >= states + base["max_partial_bytes"]
        assert info["n_passes"] >= base["n_passes"] - len(ck)
        grew += info["max_partial_bytes"] > base["max_partial_bytes"]
        checked += 1
    assert checked >= 40
    assert grew >= 1  # some checkpointed plans need more than the plain plan


def test_hbm_info_counts_the_epochs_the_checkpointed_plan_runs():
    w = Dt.make_workload("c5b")
    h = N.CircuitHandle(w.circuit)
    L = 78  # gates per hardware-efficient layer on 26 qubits
    ck = [4 * L * i for i in range(1, 5)]
    a = N.qs_hbm_info_get(h, N.QS_C64, 1)
    b = N.qs_hbm_info_get(h, N.QS_C64, 1, 0, ck)
    assert a["path"] == b["path"] == N.QS_PATH_HBM and a["tile_qubits"] == 13
    assert a["n_passes"] == N.qs_plan_info_get(h, N.QS_C64, 1)["n_segments"]
    # a checkpoint closes the epoch it falls in: never fewer epochs
    assert b["n_passes"] >= a["n_passes"]
    with pytest.raises(N.QsError) as e:  # not increasing
        N.qs_hbm_info_get(h, N.QS_C64, 1, 0, [10, 5])
    assert e.value.status == N.QS_ERR_INVALID
    with pytest.raises(N.QsError) as e:  # the fused path is not a large-state path
        N.qs_hbm_info_get(N.CircuitHandle(C.hea_ry_rz_ring(10, 2)), N.QS_C64, 4)
    assert e.value.status == N.QS_ERR_UNSUPPORTED


def test_inverse_flag_plans_the_reversed_negated_list():
    rng = np.random.default_rng(31)
    c = C.random_circuit(9, 50, rng, n_params=4, n_features=1)
    g = c.gates[::-1].copy()
    rot = np.isin(g["op"], (C.OP["RX"], C.OP["RY"], C.OP["RZ"]))
    g["scale"][rot] = -g["scale"][rot]
    rev = C.Circuit(c.n_qubits, g, c.n_params, c.n_features)
    a = N.qs_plan_info_get(N.CircuitHandle(c), N.QS_C64, 8, N.QS_FLAG_INVERSE)
    b = N.qs_plan_info_get(N.CircuitHandle(rev), N.QS_C64, 8)
    assert a == b
    assert N.qs_workspace_size(N.CircuitHandle(c), N.QS_C64, 8, N.QS_FLAG_INVERSE) == \
        N.qs_workspace_size(N.CircuitHandle(rev), N.QS_C64, 8, 0)


def test_explicit_fused_path_refuses_states_that_do_not_fit():
    """Asking for the register/LDS engine on a state it cannot hold is an
    error, never a silent switch to another path."""
    h = N.CircuitHandle(C.hea_ry_rz_ring(16, 1))
    with pytest.raises(N.QsError) as e:
        N.qs_plan_info_get(h, N.QS_C64, 1, N.QS_PATH_FUSED)
    assert e.value.status == N.QS_ERR_UNSUPPORTED
    with pytest.raises(N.QsError) as e:
        N.qs_plan_info_get(h, N.QS_C64, 1, 7)  # no such path
    assert e.value.status == N.QS_ERR_INVALID
    assert N.qs_workspace_size(h, N.QS_C64, 1, N.QS_PATH_FUSED) == 0


def test_program_layout_is_class_major():
    ub = Dt.uneven_batch(50, seed=2, n_lo=5, n_hi=8, d_lo=1, d_hi=3)
    ph = N.ProgramHandle([c for (_, _, c, _) in ub.classes],
                         [len(i) for (_, _, _, i) in ub.classes])
    so, po, eo, tot = ph.layout()
    np.testing.assert_array_equal(so, ub.state_off)
    np.testing.assert_array_equal(po, ub.param_off)
    np.testing.assert_array_equal(eo, ub.expz_off)
    assert tot[0] == ub.x.size and tot[1] == ub.params.size and tot[2] == ub.weights.size
    assert sum(len(i) for (_, _, _, i) in ub.classes) == 50


def test_workspace_sizes():
    w = Dt.make_workload("c2", 4096)
    h = N.CircuitHandle(w.circuit)
    fused = N.qs_workspace_size(h, N.QS_C64, 4096)
    info = N.qs_plan_info_get(h, N.QS_C64, 4096)
    blocks = -(-4096 // info["adj_samples_per_block"])
    # one FP32 partial sum per block and shared parameter that a rotation reads
    gs = w.circuit.gates
    rot = gs["op"] <= 2
    read = set(gs["p_w"][rot].tolist()) | set(gs["p_b"][rot].tolist())
    read.discard(-1)
    # (counted with the LDS tables bounded, so at least the launch's blocks)
    cols = max(len(read), 1)
    assert fused % (cols * 4) == 0 and fused >= blocks * cols * 4
    plain = N.qs_workspace_size(h, N.QS_C64, 4096, N.QS_PATH_PLAIN)
    assert plain == 2 * 4096 * 1024 * 8 + 4096 * w.circuit.n_gates * 8


# ------------------------------------------------ the engine program, on CPU
def _popc(x):
    return bin(int(x)).count("1")


def _run_engine_program(c, d, params, feats, psi0):
    """Executes a dumped engine program with NumPy, in the engine's own
    physical index space: read the state in under the first segment's
    layout, apply each op to physical bits, remap between segments through
    the write/read layouts, write the final state out. Independent of the
    HIP kernels; gate matrices and angles come from the oracle."""
    import oracle as O

    n, r = d["n_qubits"], d["log2_regs"]
    N, R = 1 << n, 1 << r
    B = psi0.shape[0]
    phys = np.arange(N)

    def logical(lay):
        L = np.zeros(N, dtype=np.int64)
        for bit in range(n):
            L ^= ((phys >> bit) & 1) * int(lay[bit])
        return L

    def gate_u(g):
        gt = c.gates[g]
        op = int(gt["op"])
        if op <= C.OP["RZ"]:
            return O.gate_matrix(op, O.gate_angles(gt, params, feats, B))
        return np.broadcast_to(O.gate_matrix(op), (B, 2, 2))

    lay = d["seg_lay"]
    sb = d["seg_begin"]
    cur = psi0[:, logical(lay[0][:16])]
    pat = [0xAAAAAAAA, 0xCCCCCCCC, 0xF0F0F0F0, 0xFF00FF00, 0xFFFF0000]

    def signs(rec):
        rd = d["diag"][rec]
        sign = np.ones(N)
        for p in range(N):
            k, tau = p & (R - 1), p >> r
            par = _popc(tau & int(rd[1]))
            for i in range(n - r):
                if (tau >> i) & 1:
                    par += _popc(tau & int(rd[7 + i]))
            m = int(rd[0]) ^ (0xFFFFFFFF if par & 1 else 0)
            for j in range(r):
                if _popc(tau & int(rd[2 + j])) & 1:
                    m ^= pat[j]
            if (m >> k) & 1:
                sign[p] = -1
        return sign[None, :]

    for s in range(d["n_segments"]):
        if s > 0:
            lg = np.empty_like(cur)
            lg[:, logical(lay[s - 1][16:])] = cur
            cur = lg[:, logical(lay[s][:16])]
        for o in range(sb[s], sb[s + 1]):
            kind, a, b, aux, rec = (int(v) for v in d["ops"][o])
            assert kind == 16, "every engine op is a layer op"
            assert rec == o, "the kernels read op o's record as record o"
            words = d["l1q"][rec]
            assert a == sum(1 << j for j in range(r) if words[j] >= 0)
            # a bit without a block reads the identity slot (after the fused matrices)
            assert all(words[8 + j] >= 0 for j in range(r) if words[j] < 0)
            if words[5] >= 0:
                cur = cur * signs(int(words[5]))
            for j in range(r):
                bid = int(words[j])
                if bid < 0:
                    continue
                U = np.broadcast_to(np.eye(2, dtype=np.complex128), (B, 2, 2))
                for g in d["blk_gates"][d["blk_begin"][bid]:d["blk_begin"][bid + 1]]:
                    U = gate_u(int(g)) @ U
                cur = O.apply_1q(cur, j, U)
            if words[7] >= 0:
                cur = cur * signs(int(words[7]))
    out = np.empty_like(cur)
    out[:, logical(lay[d["n_segments"] - 1][16:])] = cur
    return out


def _engine_program_case(c, seed, flags=0, B=3):
    import oracle as O

    rng = np.random.default_rng(seed)
    ps = bool(flags & N.QS_FLAG_PER_SAMPLE_PARAMS)
    params = rng.uniform(-np.pi, np.pi, (B, c.n_params) if ps else c.n_params)
    feats = rng.uniform(-1, 1, (B, c.n_features)) if c.n_features else None
    x = rng.standard_normal((B, 1 << c.n_qubits))
    psi0 = O.encode_amplitude(x, c.n_qubits)
    ref = O.run_circuit(c, params, feats, psi0)
    h = N.CircuitHandle(c)
    for adjoint in (False, True):
        d = N.qs_plan_dump(h, N.QS_C64, 64, flags, adjoint=adjoint)
        got = _run_engine_program(c, d, params, feats, psi0)
        np.testing.assert_allclose(got, ref, atol=1e-12, rtol=0)


@pytest.mark.parametrize("n", [2, 4, 5, 6, 8, 9])
def test_engine_program_executes_the_circuit(n):
    """The planner's engine program (fused blocks, sign patterns, CNOTs folded
    into remap layouts), executed on the CPU, gives the oracle's state."""
    rng = np.random.default_rng(900 + n)
    c = C.random_circuit(n, 70, rng, n_params=5, n_features=2)
    _engine_program_case(c, seed=n)
    _engine_program_case(c, seed=n, flags=N.QS_FLAG_PER_SAMPLE_PARAMS)


@pytest.mark.parametrize("kind", ["start_end", "zz", "cancel", "only"])
def test_engine_program_cnot_patterns(kind):
    _engine_program_case(cnot_pattern(7, kind), seed=3)


@pytest.mark.parametrize("key", ["c1", "c2", "c3"])
def test_engine_program_of_workloads(key):
    w = Dt.make_workload(key, 2)
    _engine_program_case(w.circuit, seed=1, B=2)


# ------------------------------------------------- dense-block plans (MFMA)
def _apply_block(psi, n, qubits, U):
    """psi [2^n] <- (U on the given qubits, local bit i = qubits[i]) psi."""
    k = len(qubits)
    t = psi.reshape([2] * n)  # axis n - 1 - q holds qubit q
    axes = [n - 1 - q for q in qubits[::-1]]  # local bit k-1 .. 0
    Ut = U.reshape([2] * (2 * k))
    out = np.tensordot(Ut, t, axes=(list(range(k, 2 * k)), axes))
    return np.moveaxis(out, list(range(k)), axes).reshape(-1)


def _check_block_plan(c, ckpt=None):
    h = N.CircuitHandle(c)
    q, b, g, k = N.qs_block_plan_export(h, N.QS_C64, 0, ckpt)
    G = c.n_gates
    assert sorted(g.tolist()) == list(range(G))  # every gate exactly once
    assert b[0] == 0 and b[-1] == G and np.all(np.diff(b) >= 1)
    for blk in range(len(q)):
        assert len(set(q[blk].tolist())) == 5 and np.all(np.diff(q[blk]) > 0)
        for gi in g[b[blk]:b[blk + 1]]:
            gt = c.gates[gi]
            assert gt["q0"] in q[blk] and (gt["q1"] < 0 or gt["q1"] in q[blk])
    # each qubit sees its gates in descriptor order
    for qq in range(c.n_qubits):
        seq = [int(x) for x in g if c.gates[x]["q0"] == qq or c.gates[x]["q1"] == qq]
        assert seq == sorted(seq), qq
    # blocks never straddle a checkpoint; the last block of each segment
    # stores its slot
    bounds = list(ckpt or []) + [G]
    seg_of = np.searchsorted(np.asarray(bounds), g, side="right")
    for blk in range(len(q)):
        assert len(set(seg_of[b[blk]:b[blk + 1]].tolist())) == 1
    assert [int(x) for x in k if x >= 0] == list(range(len(ckpt or [])))
    return q, b, g


@pytest.mark.parametrize("n,G", [(10, 120), (11, 200), (12, 90)])
def test_block_plan_executes_the_circuit(n, G):
    """The exported dense-block plan, run in NumPy block by block (each
    block's 32 x 32 unitary from the oracle's own gate matrices), equals the
    oracle's gate-by-gate run."""
    import oracle as O
    from oracle.statevector import circuit_unitary
    rng = np.random.default_rng(900 + n)
    c = C.random_circuit(n, G, rng, n_params=7, n_features=0)
    ck = sorted(set(int(v) for v in rng.integers(1, G, size=3)))
    for cks in (None, ck):
        q, b, g = _check_block_plan(c, cks)
        p = rng.uniform(-np.pi, np.pi, c.n_params)
        psi0 = O.encode_amplitude(rng.standard_normal((1, 1 << n)), n)
        ref = O.run_circuit(c, p, None, psi0)[0]
        psi = psi0[0].copy()
        for blk in range(len(q)):
            loc = {int(x): i for i, x in enumerate(q[blk])}
            rows = c.gates[g[b[blk]:b[blk + 1]]].copy()
            rows["q0"] = [loc[int(x)] for x in rows["q0"]]
            rows["q1"] = [loc[int(x)] if x >= 0 else -1 for x in rows["q1"]]
            U = circuit_unitary(C.Circuit(5, rows, c.n_params), p)
            psi = _apply_block(psi, n, [int(x) for x in q[blk]], U)
        np.testing.assert_allclose(psi, ref, atol=1e-12)


def test_block_plan_of_the_26_qubit_circuit():
    w = Dt.make_workload("c5b")
    c = w.circuit
    ck = [c.layer_end[l - 1] for l in (4, 8, 12, 16)]
    q, b, g = _check_block_plan(c)
    q2, b2, g2 = _check_block_plan(c, ck)
    # 20 layers of 78 gates on 26 qubits: about 14 gates per 5-qubit block
    assert 80 <= len(q) <= 160 and len(q2) >= len(q)
    h = N.CircuitHandle(c)
    info = N.qs_hbm_info_get(h, N.QS_C64, 1, N.QS_PATH_MFMA, ck)
    assert info["path"] == N.QS_PATH_MFMA and info["n_passes"] == len(q2)
    assert info["ws_bytes"] == N.qs_workspace_size(h, N.QS_C64, 1, N.QS_PATH_MFMA)
    assert info["ws_bytes"] >= 2 * (1 << 26) * 8


def test_block_path_refuses_what_it_does_not_run():
    h = N.CircuitHandle(C.hea_ry_rz_ring(16, 1))
    for dt, fl in [(N.QS_C128, N.QS_PATH_MFMA),
                   (N.QS_C64, N.QS_PATH_MFMA | N.QS_FLAG_PER_SAMPLE_PARAMS)]:
        with pytest.raises(N.QsError) as e:
            N.qs_plan_info_get(h, dt, 2, fl)
        assert e.value.status == N.QS_ERR_UNSUPPORTED
    # a rotation reading a feature: its angle differs per sample
    hf = N.CircuitHandle(C.reupload_ry_rz_chain(12, 2, 4))
    with pytest.raises(N.QsError):
        N.qs_plan_info_get(hf, N.QS_C64, 2, N.QS_PATH_MFMA)
    # fewer than 32 columns per state
    with pytest.raises(N.QsError):
        N.qs_plan_info_get(N.CircuitHandle(C.hea_ry_rz_ring(9, 1)), N.QS_C64, 2,
                           N.QS_PATH_MFMA)
    assert N.qs_plan_info_get(h, N.QS_C64, 2, N.QS_PATH_MFMA)["path"] == N.QS_PATH_MFMA


def test_channel_gates_validate_and_plan_only_per_call():
    """RESET / MEASURE need q1 = -1 and a feature column for their uniform;
    circuits with them are not planned by the planning calls (they run as
    engine runs between the channels) but have a workspace size."""
    base = C.hea_ry_rz_ring(5, 2)
    rng = np.random.default_rng(3)
    c = C.with_channels(base, [7, 15], rng)
    h = N.CircuitHandle(c)
    assert N.lib().qs_validate(h.ptr) == N.QS_OK
    bad = c.gates.copy()
    g = int(np.nonzero(np.isin(c.gates["op"], C.CHANNELS))[0][0])
    bad[g]["feat"] = -1
    assert N.lib().qs_validate(N.CircuitHandle(C.Circuit(5, bad, c.n_params, c.n_features)).ptr) \
        == N.QS_ERR_INVALID
    bad = c.gates.copy()
    bad[g]["q1"] = 2
    assert N.lib().qs_validate(N.CircuitHandle(C.Circuit(5, bad, c.n_params, c.n_features)).ptr) \
        == N.QS_ERR_INVALID
    with pytest.raises(N.QsError) as e:
        N.qs_plan_info_get(h, N.QS_C64, 4)
    assert e.value.status == N.QS_ERR_UNSUPPORTED
    ws = N.qs_workspace_size(h, N.QS_C64, 4)
    assert ws >= 2 * 4 * 32 * 8  # psi and lam of the batch, then partial sums
    assert N.qs_workspace_size(h, N.QS_C64, 4, N.QS_PATH_PLAIN) == 0
