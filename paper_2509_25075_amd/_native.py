"""ctypes binding of libqs.so: the calls of include/qs.h, same names.

Argument marshalling only: device tensors are passed as raw pointers, the
HIP stream is torch's current stream. Every computation happens in the HIP
library; there is no fallback. Loading fails loudly when libqs.so is absent.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs.so")

# status codes / enums (mirrors include/qs.h)
QS_OK, QS_ERR_INVALID, QS_ERR_UNSUPPORTED = 0, -1, -2
QS_ERR_WORKSPACE, QS_ERR_ZERO_NORM, QS_ERR_LAUNCH, QS_ERR_NOMEM = -3, -4, -5, -6
QS_ERR_CAPTURE, QS_ERR_NOT_PLANNED = -7, -8
QS_NOALLOC_SCRATCH_BYTES = 32 << 20
QS_C64, QS_C128 = 0, 1
QS_ENC_AMPLITUDE, QS_ENC_ZERO = 0, 1
QS_PATH_AUTO, QS_PATH_FUSED, QS_PATH_PLAIN, QS_PATH_HBM, QS_PATH_MFMA = 0, 1, 2, 3, 4
QS_FLAG_PER_SAMPLE_PARAMS = 0x100
QS_FLAG_INVERSE = 0x200

GATE_NP_DTYPE = np.dtype([
    ("op", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("p_w", "<i4"),
    ("feat", "<i4"), ("p_b", "<i4"), ("scale", "<f4"), ("flags", "<i4"),
])


class QsGate(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("q0", ctypes.c_int32),
                ("q1", ctypes.c_int32), ("p_w", ctypes.c_int32),
                ("feat", ctypes.c_int32), ("p_b", ctypes.c_int32),
                ("scale", ctypes.c_float), ("flags", ctypes.c_int32)]


class QsCircuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("n_params", ctypes.c_int32), ("n_features", ctypes.c_int32),
                ("gates", ctypes.POINTER(QsGate))]


class QsPlanInfo(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("log2_regs", ctypes.c_int32),
                ("log2_threads", ctypes.c_int32),
                ("samples_per_block", ctypes.c_int32),
                ("block_threads", ctypes.c_int32),
                ("n_segments", ctypes.c_int32), ("n_remaps", ctypes.c_int32),
                ("n_ops", ctypes.c_int32), ("lds_bytes", ctypes.c_int64),
                ("adj_log2_regs", ctypes.c_int32),
                ("adj_samples_per_block", ctypes.c_int32),
                ("adj_block_threads", ctypes.c_int32), ("n_engine_ops", ctypes.c_int32)]


class QsHbmInfo(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("n_passes", ctypes.c_int32),
                ("tile_qubits", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_partial_bytes", ctypes.c_int64), ("ws_bytes", ctypes.c_int64)]


class QsProgram(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32),
                ("circuits", ctypes.POINTER(QsCircuit)),
                ("counts", ctypes.POINTER(ctypes.c_int64))]


class QsEngineDump(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in (
        "n_qubits", "log2_regs", "n_ops", "n_segments", "n_l1q", "n_diag",
        "n_blocks", "n_block_gates")]


class QsTuneInfo(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("fwd_log2_regs", ctypes.c_int32),
                ("adj_log2_regs", ctypes.c_int32), ("tile_qubits", ctypes.c_int32),
                ("fwd_ms", ctypes.c_float), ("adj_ms", ctypes.c_float),
                ("n_candidates", ctypes.c_int32), ("fwd_samples_cap", ctypes.c_int32),
                ("adj_samples_cap", ctypes.c_int32), ("fwd_half_staging", ctypes.c_int32),
                ("adj_half_staging", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class QsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libqs.so (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_2509_25075_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    cp = ctypes.POINTER(QsCircuit)
    i32p = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "qs_version": (ctypes.c_int, []),
        "qs_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "qs_validate": (ctypes.c_int, [cp]),
        "qs_encode": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, i64,
                                     i64, ctypes.c_int, vp, i64, vp, vp, vp]),
        "qs_encode_check": (ctypes.c_int, [vp, vp]),
        "qs_forward": (ctypes.c_int, [cp, ctypes.c_int, i64, vp, vp, vp, vp,
                                      i32p, i32, vp, ctypes.c_int, vp]),
        "qs_forward_amplitude": (ctypes.c_int, [cp, ctypes.c_int, i64, vp, vp, vp,
                                                ctypes.c_int, i64, i64, vp, vp, vp,
                                                i32p, i32, vp, ctypes.c_int, vp]),
        "qs_loss_mse_z": (ctypes.c_int, [ctypes.c_int, i64, ctypes.c_int, vp, vp, vp, vp,
                                         vp]),
        "qs_train_step_mse": (ctypes.c_int, [cp, ctypes.c_int, i64, vp, vp, vp, ctypes.c_int,
                                             i64, i64, vp, vp, ctypes.c_int, vp, vp, vp, vp,
                                             vp, sz, ctypes.c_int, vp]),
        "qs_train_workspace_size": (sz, [cp, ctypes.c_int, i64, ctypes.c_int]),
        "qs_workspace_size": (sz, [cp, ctypes.c_int, i64, ctypes.c_int]),
        "qs_adjoint_backward": (ctypes.c_int, [cp, ctypes.c_int, i64, vp, vp, vp,
                                               vp, vp, vp, vp, i32p, i32, vp, vp,
                                               sz, ctypes.c_int, vp]),
        "qs_adjoint_backward_noalloc": (ctypes.c_int, [cp, ctypes.c_int, i64, vp, vp, vp,
                                                       vp, vp, vp, vp, i32p, i32, vp,
                                                       ctypes.c_int, vp]),
        "qs_expz": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, i64, vp, vp, vp]),
        "qs_fidelity_reset": (ctypes.c_int, [ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, i64, vp, vp, vp, vp,
                                             vp, vp, vp]),
        "qs_fidelity_postselect": (ctypes.c_int, [ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, i64, vp, vp, vp, vp,
                                                  vp, vp, vp]),
        "qs_fidelity_trajectory": (ctypes.c_int, [ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, i64, vp, vp, vp, vp,
                                                  vp, vp, vp, vp, vp]),
        "qs_plan_info_get": (ctypes.c_int, [cp, ctypes.c_int, i64, ctypes.c_int,
                                            ctypes.POINTER(QsPlanInfo)]),
        "qs_hbm_info_get": (ctypes.c_int, [cp, ctypes.c_int, i64, ctypes.c_int, i32p,
                                           i32, ctypes.POINTER(QsHbmInfo)]),
        "qs_block_plan_export": (ctypes.c_int, [cp, ctypes.c_int, ctypes.c_int, i32p, i32,
                                                i32p, vp, vp, vp, vp]),
        "qs_plan_export": (ctypes.c_int, [cp, ctypes.c_int, i64, ctypes.c_int,
                                          ctypes.POINTER(QsPlanInfo), vp, vp, vp]),
        "qs_program_layout": (ctypes.c_int, [ctypes.POINTER(QsProgram), vp, vp, vp, vp]),
        "qs_program_encode": (ctypes.c_int, [ctypes.POINTER(QsProgram), ctypes.c_int, vp,
                                             ctypes.c_int, vp, vp, vp]),
        "qs_program_forward": (ctypes.c_int, [ctypes.POINTER(QsProgram), ctypes.c_int, vp,
                                              vp, vp, vp]),
        "qs_program_adjoint": (ctypes.c_int, [ctypes.POINTER(QsProgram), ctypes.c_int, vp,
                                              vp, vp, vp, vp]),
        "qs_autotune": (ctypes.c_int, [cp, ctypes.c_int, i64, ctypes.c_int, vp,
                                       ctypes.POINTER(QsTuneInfo)]),
        "qs_plan_dump": (ctypes.c_int, [cp, ctypes.c_int, i64, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(QsEngineDump), vp, vp, vp, vp, vp,
                                        vp, vp]),
        "qs_shutdown": (None, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().qs_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != QS_OK:
        raise QsError(status, where)


class CircuitHandle:
    """A circuit descriptor in the C layout, kept alive for ctypes calls.

    Built from any object with ``n_qubits``, ``gates`` (a structured array in
    the descriptor layout), ``n_params`` and ``n_features``.
    """

    def __init__(self, circuit):
        g = np.ascontiguousarray(np.asarray(circuit.gates).astype(GATE_NP_DTYPE))
        self._gates = g
        self.n_qubits = int(circuit.n_qubits)
        self.n_params = int(circuit.n_params)
        self.n_features = int(circuit.n_features)
        self.n_gates = int(g.shape[0])
        self.c = QsCircuit(self.n_qubits, self.n_gates, self.n_params,
                           self.n_features,
                           ctypes.cast(g.ctypes.data, ctypes.POINTER(QsGate)))

    @property
    def ptr(self):
        return ctypes.byref(self.c)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ckpt_arr(ckpt_gates):
    if not ckpt_gates:
        return None, 0, None
    arr = (ctypes.c_int32 * len(ckpt_gates))(*[int(v) for v in ckpt_gates])
    return arr, len(ckpt_gates), arr


# ------------------------------------------------------------------- calls
def qs_version() -> int:
    return lib().qs_version()


def qs_validate(h: CircuitHandle) -> int:
    return lib().qs_validate(h.ptr)


def qs_encode(enc: int, dtype: int, n_qubits: int, x, state, bad_rows=None,
              stream=None):
    """x: [B, D] float32/float64 device tensor (ignored for QS_ENC_ZERO);
    state: [B, 2^n] complex64/complex128 device tensor (written)."""
    B = state.shape[0]
    if enc == QS_ENC_AMPLITUDE:
        D, xs, f64 = x.shape[1], x.stride(0), int(x.dtype.itemsize == 8)
    else:
        D, xs, f64 = 0, 0, 0
    _check(lib().qs_encode(enc, dtype, n_qubits, B, D, f64, _ptr(x), xs,
                           _ptr(state), _ptr(bad_rows), _stream(stream)),
           "qs_encode")


def qs_encode_check(bad_rows, stream=None):
    """Waits for the stream and raises QsError(QS_ERR_ZERO_NORM) when the
    bad-row counter of earlier encodes is non-zero."""
    _check(lib().qs_encode_check(_ptr(bad_rows), _stream(stream)), "qs_encode_check")


def qs_forward(h: CircuitHandle, dtype: int, params, feats, state, expz=None,
               ckpt_gates=None, ckpt=None, flags: int = 0, stream=None):
    arr, n_ck, keep = _ckpt_arr(ckpt_gates)
    _check(lib().qs_forward(h.ptr, dtype, state.shape[0], _ptr(params),
                            _ptr(feats), _ptr(state), _ptr(expz), arr, n_ck,
                            _ptr(ckpt), flags, _stream(stream)), "qs_forward")
    del keep


def qs_forward_amplitude(h: CircuitHandle, dtype: int, params, feats, x, state,
                         expz=None, bad_rows=None, ckpt_gates=None, ckpt=None,
                         flags: int = 0, stream=None):
    """x: [B, D] float32/float64 device tensor (row stride may exceed D);
    state: [B, 2^n] complex device tensor, receives the final state."""
    arr, n_ck, keep = _ckpt_arr(ckpt_gates)
    D, xs, f64 = x.shape[1], x.stride(0), int(x.dtype.itemsize == 8)
    _check(lib().qs_forward_amplitude(h.ptr, dtype, state.shape[0], _ptr(params),
                                      _ptr(feats), _ptr(x), f64, D, xs, _ptr(bad_rows),
                                      _ptr(state), _ptr(expz), arr, n_ck, _ptr(ckpt),
                                      flags, _stream(stream)), "qs_forward_amplitude")
    del keep


def qs_loss_mse_z(q: int, expz, y, dexpz=None, loss=None, stream=None):
    """expz: [B, n] float64, y: [B] float64; dexpz [B, n] and loss [1] float64
    device outputs (either may be None)."""
    B, n = expz.shape
    _check(lib().qs_loss_mse_z(n, B, q, _ptr(expz), _ptr(y), _ptr(dexpz), _ptr(loss),
                               _stream(stream)), "qs_loss_mse_z")


def qs_train_workspace_size(h: CircuitHandle, dtype: int, B: int, flags: int = 0) -> int:
    return int(lib().qs_train_workspace_size(h.ptr, dtype, B, flags))


def qs_train_step_mse(h: CircuitHandle, dtype: int, params, feats, x, y, q: int, loss,
                      grad_params, ws, expz=None, grad_feats=None, bad_rows=None,
                      B: int | None = None, flags: int = 0, stream=None):
    """One-launch training step (see include/qs.h). x: [B, D] float32 device
    tensor or None (start from |0...0>, then B must be given); y [B] float64;
    loss [1] float64; ws uint8 of qs_train_workspace_size bytes."""
    if x is not None:
        B, D, xs, f64 = x.shape[0], x.shape[1], x.stride(0), int(x.dtype.itemsize == 8)
    else:
        D, xs, f64 = 0, 0, 0
    _check(lib().qs_train_step_mse(h.ptr, dtype, B, _ptr(params), _ptr(feats), _ptr(x), f64,
                                   D, xs, _ptr(bad_rows), _ptr(y), q, _ptr(expz), _ptr(loss),
                                   _ptr(grad_params), _ptr(grad_feats), _ptr(ws), ws.numel(),
                                   flags, _stream(stream)), "qs_train_step_mse")


def qs_workspace_size(h: CircuitHandle, dtype: int, B: int, flags: int = 0) -> int:
    return int(lib().qs_workspace_size(h.ptr, dtype, B, flags))


def qs_adjoint_backward(h: CircuitHandle, dtype: int, params, feats, state,
                        dexpz=None, dstate=None, grad_params=None,
                        grad_feats=None, ckpt_gates=None, ckpt=None, ws=None,
                        flags: int = 0, stream=None):
    arr, n_ck, keep = _ckpt_arr(ckpt_gates)
    ws_bytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(lib().qs_adjoint_backward(
        h.ptr, dtype, state.shape[0], _ptr(params), _ptr(feats), _ptr(state),
        _ptr(dexpz), _ptr(dstate), _ptr(grad_params), _ptr(grad_feats), arr,
        n_ck, _ptr(ckpt), _ptr(ws), ws_bytes, flags, _stream(stream)),
        "qs_adjoint_backward")
    del keep


def qs_adjoint_backward_noalloc(h: CircuitHandle, dtype: int, params, feats, state,
                                dexpz=None, dstate=None, grad_params=None,
                                grad_feats=None, ckpt_gates=None, ckpt=None,
                                flags: int = 0, stream=None):
    """qs_adjoint_backward with the library's own device scratch array in
    place of a workspace (no device allocation; the shape must be planned)."""
    arr, n_ck, keep = _ckpt_arr(ckpt_gates)
    _check(lib().qs_adjoint_backward_noalloc(
        h.ptr, dtype, state.shape[0], _ptr(params), _ptr(feats), _ptr(state),
        _ptr(dexpz), _ptr(dstate), _ptr(grad_params), _ptr(grad_feats), arr,
        n_ck, _ptr(ckpt), flags, _stream(stream)), "qs_adjoint_backward_noalloc")
    del keep


def qs_expz(dtype: int, n_qubits: int, state, expz, stream=None):
    _check(lib().qs_expz(dtype, n_qubits, state.shape[0], _ptr(state),
                         _ptr(expz), _stream(stream)), "qs_expz")


def qs_fidelity_reset(dtype: int, n_qubits: int, n_trash: int, psi, chi, fid,
                      dfid=None, lam_psi=None, lam_chi=None, stream=None):
    _check(lib().qs_fidelity_reset(dtype, n_qubits, n_trash, psi.shape[0],
                                   _ptr(psi), _ptr(chi), _ptr(fid), _ptr(dfid),
                                   _ptr(lam_psi), _ptr(lam_chi),
                                   _stream(stream)), "qs_fidelity_reset")


def qs_fidelity_postselect(dtype: int, n_qubits: int, n_trash: int, psi, chi, fid,
                           dfid=None, lam_psi=None, lam_chi=None, stream=None):
    _check(lib().qs_fidelity_postselect(dtype, n_qubits, n_trash, psi.shape[0],
                                        _ptr(psi), _ptr(chi), _ptr(fid), _ptr(dfid),
                                        _ptr(lam_psi), _ptr(lam_chi),
                                        _stream(stream)), "qs_fidelity_postselect")


def qs_fidelity_trajectory(dtype: int, n_qubits: int, n_trash: int, psi, chi, u, fid,
                           outcome=None, dfid=None, lam_psi=None, lam_chi=None,
                           stream=None):
    _check(lib().qs_fidelity_trajectory(dtype, n_qubits, n_trash, psi.shape[0],
                                        _ptr(psi), _ptr(chi), _ptr(u), _ptr(fid),
                                        _ptr(outcome), _ptr(dfid), _ptr(lam_psi),
                                        _ptr(lam_chi), _stream(stream)),
           "qs_fidelity_trajectory")


def qs_hbm_info_get(h: CircuitHandle, dtype: int, B: int, flags: int = 0,
                    ckpt_gates=None) -> dict:
    arr, n, _ = _ckpt_arr(ckpt_gates)
    info = QsHbmInfo()
    _check(lib().qs_hbm_info_get(h.ptr, dtype, B, flags, arr, n, ctypes.byref(info)),
           "qs_hbm_info_get")
    return {k: getattr(info, k) for k, _ in QsHbmInfo._fields_}


def qs_block_plan_export(h: CircuitHandle, dtype: int = QS_C64, flags: int = 0,
                         ckpt_gates=None):
    """The dense-block plan: (qubits [nb, 5], begin [nb + 1], gates [G],
    ckpt [nb]) as int32 arrays."""
    arr, n, _ = _ckpt_arr(ckpt_gates)
    nb = ctypes.c_int32(0)
    L = lib()
    _check(L.qs_block_plan_export(h.ptr, dtype, flags, arr, n, ctypes.byref(nb),
                                  None, None, None, None), "qs_block_plan_export")
    q = np.zeros((nb.value, 5), np.int32)
    b = np.zeros(nb.value + 1, np.int32)
    g = np.zeros(max(h.n_gates, 1), np.int32)
    k = np.zeros(nb.value, np.int32)
    _check(L.qs_block_plan_export(h.ptr, dtype, flags, arr, n, ctypes.byref(nb),
                                  q.ctypes.data, b.ctypes.data, g.ctypes.data,
                                  k.ctypes.data), "qs_block_plan_export")
    return q, b, g[:h.n_gates], k


def qs_plan_info_get(h: CircuitHandle, dtype: int, B: int, flags: int = 0) -> dict:
    info = QsPlanInfo()
    _check(lib().qs_plan_info_get(h.ptr, dtype, B, flags, ctypes.byref(info)),
           "qs_plan_info_get")
    return {k: getattr(info, k) for k, _ in QsPlanInfo._fields_}


def qs_plan_export(h: CircuitHandle, dtype: int, B: int, flags: int = 0):
    """Host-only plan export: (info dict, ops [n_ops, 4] int32,
    seg_begin [nseg + 1] int32, seg_map [nseg, 16] uint8)."""
    info = QsPlanInfo()
    _check(lib().qs_plan_export(h.ptr, dtype, B, flags, ctypes.byref(info),
                                None, None, None), "qs_plan_export")
    ops = np.zeros((info.n_ops, 4), dtype=np.int32)
    sb = np.zeros(info.n_segments + 1, dtype=np.int32)
    sm = np.zeros((info.n_segments, 16), dtype=np.uint8)
    _check(lib().qs_plan_export(h.ptr, dtype, B, flags, ctypes.byref(info),
                                ops.ctypes.data, sb.ctypes.data, sm.ctypes.data),
           "qs_plan_export")
    return ({k: getattr(info, k) for k, _ in QsPlanInfo._fields_}, ops, sb, sm)


class ProgramHandle:
    """An uneven batch in the C layout: classes (circuit, count)."""

    def __init__(self, circuits, counts):
        self.handles = [CircuitHandle(c) for c in circuits]
        arr = (QsCircuit * len(circuits))(*[h.c for h in self.handles])
        self._arr = arr
        self._counts = (ctypes.c_int64 * len(counts))(*[int(v) for v in counts])
        self.p = QsProgram(len(circuits), arr, self._counts)

    @property
    def ptr(self):
        return ctypes.byref(self.p)

    def layout(self):
        k = self.p.n_classes
        so, po, eo = (np.zeros(k, np.int64) for _ in range(3))
        tot = np.zeros(3, np.int64)
        _check(lib().qs_program_layout(self.ptr, so.ctypes.data, po.ctypes.data,
                                       eo.ctypes.data, tot.ctypes.data), "qs_program_layout")
        return so, po, eo, tot


def qs_program_encode(ph: ProgramHandle, dtype: int, x, states, bad_rows=None, stream=None):
    _check(lib().qs_program_encode(ph.ptr, dtype, _ptr(x), int(x.dtype.itemsize == 8),
                                   _ptr(states), _ptr(bad_rows), _stream(stream)),
           "qs_program_encode")


def qs_program_forward(ph: ProgramHandle, dtype: int, params, states, expz=None,
                       stream=None):
    _check(lib().qs_program_forward(ph.ptr, dtype, _ptr(params), _ptr(states),
                                    _ptr(expz), _stream(stream)), "qs_program_forward")


def qs_program_adjoint(ph: ProgramHandle, dtype: int, params, states, dexpz,
                       grad_params, stream=None):
    _check(lib().qs_program_adjoint(ph.ptr, dtype, _ptr(params), _ptr(states),
                                    _ptr(dexpz), _ptr(grad_params), _stream(stream)),
           "qs_program_adjoint")


def qs_autotune(h: CircuitHandle, dtype: int, B: int, flags: int = 0, stream=None) -> dict:
    info = QsTuneInfo()
    _check(lib().qs_autotune(h.ptr, dtype, B, flags, _stream(stream), ctypes.byref(info)),
           "qs_autotune")
    return {k: getattr(info, k) for k, _ in QsTuneInfo._fields_}


def qs_plan_dump(h: CircuitHandle, dtype: int, B: int, flags: int = 0,
                 adjoint: bool = False) -> dict:
    """Host-only dump of the engine program (see include/qs.h)."""
    info = QsEngineDump()
    args = (h.ptr, dtype, B, flags, int(adjoint), ctypes.byref(info))
    _check(lib().qs_plan_dump(*args, None, None, None, None, None, None, None),
           "qs_plan_dump")
    d = {k: getattr(info, k) for k, _ in QsEngineDump._fields_}
    arr = {
        "ops": np.zeros((max(d["n_ops"], 1), 5), np.int32),
        "seg_begin": np.zeros(d["n_segments"] + 1, np.int32),
        "seg_lay": np.zeros((max(d["n_segments"], 1), 32), np.uint16),
        "l1q": np.zeros((max(d["n_l1q"], 1), 16), np.int32),
        "diag": np.zeros((max(d["n_diag"], 1), 24), np.uint32),
        "blk_begin": np.zeros(d["n_blocks"] + 1, np.int32),
        "blk_gates": np.zeros(max(d["n_block_gates"], 1), np.int32),
    }
    _check(lib().qs_plan_dump(*args, *(a.ctypes.data_as(ctypes.c_void_p) for a in (
        arr["ops"], arr["seg_begin"], arr["seg_lay"], arr["l1q"], arr["diag"],
        arr["blk_begin"], arr["blk_gates"]))), "qs_plan_dump")
    arr["ops"] = arr["ops"][:d["n_ops"]]
    d.update(arr)
    return d


def qs_shutdown():
    lib().qs_shutdown()
