"""Torch-facing layer over the HIP library: device buffers, the autograd
Function, and one training step of a workload.

PyTorch supplies device memory and the stream; every step of the state
simulation (encoding, gate sweep, readout, adjoint, fidelity) runs in
libqs.so. The loss and its upstream gradient dL/d<Z> are the only arithmetic
done in torch, on the GPU.
"""

from __future__ import annotations

from dataclasses import dataclass

import torch

from . import _native as N

_DT = {
    "c64": (N.QS_C64, torch.complex64, torch.float32),
    "c128": (N.QS_C128, torch.complex128, torch.float64),
}


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2509_25075_amd needs a ROCm GPU (no CPU fallback)")
    N.lib()


class Simulator:
    """One circuit on one dtype: encode, forward, adjoint on device tensors."""

    def __init__(self, circuit, dtype: str = "c64", flags: int = 0):
        require_gpu()
        self.circuit = circuit
        self.h = N.CircuitHandle(circuit)
        self.dtype = dtype
        self.qs_dtype, self.cdtype, self.rdtype = _DT[dtype]
        self.flags = flags
        self.n = self.h.n_qubits

    # -------------------------------------------------------------- states
    def empty_state(self, B: int, device="cuda"):
        return torch.empty((B, 1 << self.n), dtype=self.cdtype, device=device)

    def encode_amplitude(self, x, out=None):
        out = self.empty_state(x.shape[0], x.device) if out is None else out
        N.qs_encode(N.QS_ENC_AMPLITUDE, self.qs_dtype, self.n, x, out)
        return out

    def zero_state(self, B: int, device="cuda", out=None):
        out = self.empty_state(B, device) if out is None else out
        N.qs_encode(N.QS_ENC_ZERO, self.qs_dtype, self.n, None, out)
        return out

    # ------------------------------------------------------------- sweeps
    def forward(self, params, feats, state, want_expz=True, ckpt_gates=None,
                ckpt=None, flags=None, x=None, bad_rows=None):
        """In-place forward on ``state``; returns <Z> [B, n] (float64) or None.
        With ``x`` ([B, D] real amplitude inputs), the sweep starts from their
        amplitude encoding instead (one call: qs_forward_amplitude) and
        ``state`` only receives the final state."""
        B = state.shape[0]
        expz = torch.empty((B, self.n), dtype=torch.float64,
                           device=state.device) if want_expz else None
        fl = self.flags if flags is None else flags
        if x is None:
            N.qs_forward(self.h, self.qs_dtype, params, feats, state, expz,
                         ckpt_gates, ckpt, fl)
        else:
            N.qs_forward_amplitude(self.h, self.qs_dtype, params, feats, x, state, expz,
                                   bad_rows, ckpt_gates, ckpt, fl)
        return expz

    def workspace(self, B: int, device="cuda", flags=None):
        nbytes = N.qs_workspace_size(self.h, self.qs_dtype, B,
                                     self.flags if flags is None else flags)
        return torch.empty(max(nbytes, 8), dtype=torch.uint8, device=device)

    def adjoint(self, params, feats, state, dexpz=None, dstate=None, ws=None,
                ckpt_gates=None, ckpt=None, flags=None, want_feat_grad=True):
        """Returns (grad_params float64, grad_feats float64 or None)."""
        fl = self.flags if flags is None else flags
        B = state.shape[0]
        dev = state.device
        per_sample = bool(fl & N.QS_FLAG_PER_SAMPLE_PARAMS)
        gp = torch.empty((B, self.h.n_params) if per_sample else (self.h.n_params,),
                         dtype=torch.float64, device=dev)
        gf = None
        if self.h.n_features and want_feat_grad:
            gf = torch.empty((B, self.h.n_features), dtype=torch.float64, device=dev)
        ws = self.workspace(B, dev, fl) if ws is None else ws
        N.qs_adjoint_backward(self.h, self.qs_dtype, params, feats, state,
                              dexpz=dexpz, dstate=dstate, grad_params=gp,
                              grad_feats=gf, ckpt_gates=ckpt_gates, ckpt=ckpt,
                              ws=ws, flags=fl)
        return gp, gf

    def plan_info(self, B: int, flags=None) -> dict:
        return N.qs_plan_info_get(self.h, self.qs_dtype, B,
                                  self.flags if flags is None else flags)


class CircuitExpZ(torch.autograd.Function):
    """<Z_q>_b of circuit(params, feats) applied to a fixed encoded state,
    differentiable in params and feats through the library's adjoint."""

    @staticmethod
    def forward(ctx, params, feats, state0, sim: Simulator):
        state = state0.clone()
        expz = sim.forward(params.detach(), None if feats is None else feats.detach(),
                           state)
        ctx.sim = sim
        ctx.has_feats = feats is not None
        ctx.save_for_backward(params, feats if feats is not None else params, state)
        return expz

    @staticmethod
    def backward(ctx, gexpz):
        params, feats, state = ctx.saved_tensors
        feats = feats if ctx.has_feats else None
        gp, gf = ctx.sim.adjoint(params.detach(),
                                 None if feats is None else feats.detach(), state,
                                 dexpz=gexpz.contiguous().to(torch.float64))
        gp = gp.to(params.dtype)
        gf = None if gf is None else gf.to(feats.dtype)
        return gp, gf, None, None


def expz(params, feats, state0, sim: Simulator):
    return CircuitExpZ.apply(params, feats, state0, sim)


_FIDELITY = {"reset": "qs_fidelity_reset", "postselect": "qs_fidelity_postselect",
             "trajectory": "qs_fidelity_trajectory"}


class AutoencoderFidelity(torch.autograd.Function):
    """Per-sample autoencoder fidelity F_b of an encoder U(params_enc) and a
    decoder V(params_dec)^dagger on the encoded inputs state0, with the
    n_trash top qubits reset ("reset"), measured with only the all-zero
    outcome kept ("postselect"), or reset along one trajectory drawn by the
    uniforms u ("trajectory"); differentiable in both parameter sets through
    the library's fidelity cotangents and adjoint."""

    @staticmethod
    def forward(ctx, params_enc, params_dec, state0, enc: Simulator, dec: Simulator,
                n_trash: int, kind: str = "reset", u=None):
        psi = state0.clone()
        chi = state0.clone()
        enc.forward(params_enc.detach(), None, psi, want_expz=False)
        dec.forward(params_dec.detach(), None, chi, want_expz=False)
        fid = torch.empty(state0.shape[0], dtype=torch.float64, device=state0.device)
        ctx.enc, ctx.dec, ctx.n_trash, ctx.kind = enc, dec, n_trash, kind
        ctx.save_for_backward(params_enc, params_dec, psi, chi,
                              u if u is not None else fid)
        _fidelity_call(enc, kind, n_trash, psi, chi, fid, u=u)
        return fid

    @staticmethod
    def backward(ctx, gfid):
        params_enc, params_dec, psi, chi, u = ctx.saved_tensors
        u = u if ctx.kind == "trajectory" else None
        fid = torch.empty(psi.shape[0], dtype=torch.float64, device=psi.device)
        lam_psi = torch.empty_like(psi)
        lam_chi = torch.empty_like(chi)
        _fidelity_call(ctx.enc, ctx.kind, ctx.n_trash, psi, chi, fid, u=u,
                       dfid=gfid.contiguous().to(torch.float64), lam_psi=lam_psi,
                       lam_chi=lam_chi)
        ge, _ = ctx.enc.adjoint(params_enc.detach(), None, psi, dstate=lam_psi)
        gd, _ = ctx.dec.adjoint(params_dec.detach(), None, chi, dstate=lam_chi)
        return ge.to(params_enc.dtype), gd.to(params_dec.dtype), None, None, None, None, \
            None, None


def _fidelity_call(sim: Simulator, kind, n_trash, psi, chi, fid, u=None, dfid=None,
                   lam_psi=None, lam_chi=None):
    if kind == "trajectory":
        N.qs_fidelity_trajectory(sim.qs_dtype, sim.n, n_trash, psi, chi, u, fid, None,
                                 dfid, lam_psi, lam_chi)
    else:
        getattr(N, _FIDELITY[kind])(sim.qs_dtype, sim.n, n_trash, psi, chi, fid, dfid,
                                    lam_psi, lam_chi)


def autoencoder_fidelity(params_enc, params_dec, state0, enc: Simulator, dec: Simulator,
                         n_trash: int, kind: str = "reset", u=None):
    return AutoencoderFidelity.apply(params_enc, params_dec, state0, enc, dec, n_trash,
                                     kind, u)


# ---------------------------------------------------------------- workloads
@dataclass
class DeviceWorkload:
    """A workload's inputs resident on the GPU, plus preallocated buffers."""
    w: object
    sim: Simulator
    sim_dec: Simulator | None
    x: torch.Tensor | None
    feats: torch.Tensor | None
    params: torch.Tensor
    params_dec: torch.Tensor | None
    labels: torch.Tensor | None
    weights: torch.Tensor | None
    state: torch.Tensor
    state_dec: torch.Tensor | None
    ws: torch.Tensor
    ws_dec: torch.Tensor | None
    flags: int
    ckpt_gates: list | None = None   # gate counts after which psi is stored
    ckpt: torch.Tensor | None = None  # [n_ckpt, B, 2^n] stored states
    dz: torch.Tensor | None = None    # [B, n] float64 upstream gradient buffer
    u: torch.Tensor | None = None     # [B] float64 trajectory uniforms
    loss_buf: torch.Tensor | None = None  # [1] float64 loss of the last step
    dfid: torch.Tensor | None = None  # [B] float64 dL/dF_b = -1/B (fidelity losses)
    train_ws: torch.Tensor | None = None  # workspace of the one-launch training step
    # Run MSE steps as one launch (qs_train_step_mse) where the library has
    # that kernel: on the 10-qubit batch it measured 9 % faster than the
    # forward, loss and adjoint launches it replaces, and it never writes the
    # [B][2^n] state to HBM. False forces the separate launches.
    one_launch: bool = True


def to_device(w, flags: int = 0, device="cuda", ckpt_every_layers: int = 0,
              traj_u=None, one_launch: bool = True) -> DeviceWorkload:
    """``traj_u``: [B] uniforms in [0, 1) that draw the measurement outcome of
    each sample's reset-channel trajectory (loss "fidelity_trajectory")."""
    if w.loss == "fidelity_trajectory" and traj_u is None:
        raise ValueError("the trajectory loss needs its uniforms (traj_u)")
    sim = Simulator(w.circuit, w.dtype, flags)
    rd = sim.rdtype
    B = w.batch
    t = lambda a, dt=rd: None if a is None else torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
    sim_dec = Simulator(w.decoder, w.dtype, flags) if w.decoder is not None else None
    state = sim.empty_state(B, device)
    ckpt_gates, ckpt = None, None
    if ckpt_every_layers and w.decoder is None:
        ends = w.circuit.layer_end
        ckpt_gates = [ends[l - 1] for l in range(ckpt_every_layers, len(ends),
                                                 ckpt_every_layers)]
        if ckpt_gates:
            ckpt = torch.empty((len(ckpt_gates), B, 1 << w.n_qubits),
                               dtype=sim.cdtype, device=device)
        else:
            ckpt_gates = None
    # Upstream gradient dL/d<Z>: MSE on qubit 0 writes column 0 each step
    # (the others stay zero); a weighted sum has a constant one.
    dz, dfid = None, None
    if w.loss == "mse_z0":
        dz = torch.zeros((B, w.n_qubits), dtype=torch.float64, device=device)
    elif w.loss == "weighted_z":
        dz = t(w.weights, torch.float64)[None, :].expand(B, w.n_qubits).contiguous()
    elif w.loss.startswith("fidelity"):
        dfid = torch.full((B,), -1.0 / B, dtype=torch.float64, device=device)
    return DeviceWorkload(
        w=w, sim=sim, sim_dec=sim_dec, x=t(w.x), feats=t(w.feats),
        params=t(w.params), params_dec=t(w.params_dec),
        labels=t(w.labels, torch.float64), weights=t(w.weights, torch.float64),
        state=state, state_dec=sim.empty_state(B, device) if sim_dec else None,
        ws=sim.workspace(B, device, flags),
        ws_dec=sim_dec.workspace(B, device, flags) if sim_dec else None,
        flags=flags, ckpt_gates=ckpt_gates, ckpt=ckpt, dz=dz,
        u=t(traj_u, torch.float64) if w.loss == "fidelity_trajectory" else None,
        loss_buf=torch.zeros(1, dtype=torch.float64, device=device), dfid=dfid,
        one_launch=one_launch)


def train_step_runs(d: DeviceWorkload) -> bool:
    """Whether step() runs the workload's training step as one launch
    (qs_train_step_mse): not switched off (one_launch), the MSE loss, no
    checkpoints, and a shape the library has that kernel for."""
    return (d.one_launch and d.w.loss == "mse_z0" and not d.ckpt_gates and
            N.qs_train_workspace_size(d.sim.h, d.sim.qs_dtype, d.w.batch, d.flags) > 0)


def step(d: DeviceWorkload, backward: bool = True) -> dict:
    """One pass of the whole path: encode, forward sweep, readout, loss,
    adjoint backward. Returns the device tensors it produced."""
    w, sim = d.w, d.sim
    B = w.batch
    # Amplitude inputs are encoded by the forward call itself.
    x = d.x if w.encoding == "amplitude" else None
    out = {}
    if w.loss in ("fidelity_reset", "fidelity_postselect", "fidelity_trajectory"):
        if x is None:
            sim.zero_state(B, d.state.device, out=d.state)
            sim.zero_state(B, d.state.device, out=d.state_dec)
        sim.forward(d.params, d.feats, d.state, want_expz=False, x=x)
        d.sim_dec.forward(d.params_dec, d.feats, d.state_dec, want_expz=False, x=x)
        fid = torch.empty(B, dtype=torch.float64, device=d.state.device)
        dfid = d.dfid
        lam_psi = torch.empty_like(d.state)
        lam_chi = torch.empty_like(d.state)
        if w.loss == "fidelity_trajectory":
            N.qs_fidelity_trajectory(sim.qs_dtype, sim.n, w.n_trash, d.state, d.state_dec,
                                     d.u, fid, None, dfid if backward else None,
                                     lam_psi if backward else None,
                                     lam_chi if backward else None)
        else:
            fn = (N.qs_fidelity_reset if w.loss == "fidelity_reset"
                  else N.qs_fidelity_postselect)
            fn(sim.qs_dtype, sim.n, w.n_trash, d.state, d.state_dec,
               fid, dfid if backward else None,
               lam_psi if backward else None,
               lam_chi if backward else None)
        out["fid"] = fid
        out["loss"] = 1.0 - fid.mean()
        if backward:
            out["grad_params"], _ = sim.adjoint(d.params, d.feats, d.state,
                                                dstate=lam_psi, ws=d.ws)
            out["grad_params_dec"], _ = d.sim_dec.adjoint(
                d.params_dec, d.feats, d.state_dec, dstate=lam_chi, ws=d.ws_dec)
        return out
    if backward and train_step_runs(d):
        # The whole step in one engine launch where the library has that
        # kernel for the tuned shape (qs_train_step_mse), else three calls.
        need = N.qs_train_workspace_size(sim.h, sim.qs_dtype, B, d.flags)
        if need > 0:
            if d.train_ws is None or d.train_ws.numel() < need:
                d.train_ws = torch.empty(need, dtype=torch.uint8, device=d.state.device)
            dev = d.state.device
            z = torch.empty((B, sim.n), dtype=torch.float64, device=dev)
            gp = torch.empty(sim.h.n_params, dtype=torch.float64, device=dev)
            gf = (torch.empty((B, sim.h.n_features), dtype=torch.float64, device=dev)
                  if sim.h.n_features else None)
            N.qs_train_step_mse(sim.h, sim.qs_dtype, d.params, d.feats, x, d.labels, 0,
                                d.loss_buf, gp, d.train_ws, expz=z, grad_feats=gf, B=B,
                                flags=d.flags)
            out.update(expz=z, loss=d.loss_buf[0], grad_params=gp)
            if gf is not None:
                out["grad_feats"] = gf
            return out
    if x is None:
        sim.zero_state(B, d.state.device, out=d.state)
    z = sim.forward(d.params, d.feats, d.state, want_expz=True,
                    ckpt_gates=d.ckpt_gates, ckpt=d.ckpt, x=x)
    out["expz"] = z
    if w.loss == "none" or not backward:
        return out
    dz = d.dz
    if w.loss == "mse_z0":
        N.qs_loss_mse_z(0, z, d.labels, dexpz=dz, loss=d.loss_buf)
        out["loss"] = d.loss_buf[0]
    elif w.loss == "weighted_z":
        out["loss"] = (z * d.weights[None, :]).sum()
    else:
        raise ValueError(w.loss)
    gp, gf = sim.adjoint(d.params, d.feats, d.state, dexpz=dz, ws=d.ws,
                         ckpt_gates=d.ckpt_gates, ckpt=d.ckpt)
    out["grad_params"] = gp
    if gf is not None:
        out["grad_feats"] = gf
    return out


# ------------------------------------------------------------- uneven batch
class UnevenDevice:
    """An uneven batch resident on the GPU: packed inputs, parameters, readout
    weights, states, <Z> and gradient buffers; one step = program encode,
    persistent forward (with FP64 readout), loss sum_q g_q <Z_q>, persistent
    adjoint."""

    def __init__(self, ub, dtype: str = "c64", device="cuda"):
        require_gpu()
        self.ub = ub
        self.dtype = dtype
        self.qs_dtype, self.cdtype, self.rdtype = _DT[dtype]
        self.ph = N.ProgramHandle([c for (_, _, c, _) in ub.classes],
                                  [len(idx) for (_, _, _, idx) in ub.classes])
        so, po, eo, tot = self.ph.layout()
        assert (so == ub.state_off).all() and (po == ub.param_off).all() \
            and (eo == ub.expz_off).all()
        self.x = torch.as_tensor(ub.x).to(device=device, dtype=self.rdtype)
        self.params = torch.as_tensor(ub.params).to(device=device, dtype=self.rdtype)
        self.weights = torch.as_tensor(ub.weights).to(device=device, dtype=torch.float64)
        self.states = torch.empty(int(tot[0]), dtype=self.cdtype, device=device)
        self.expz = torch.empty(int(tot[2]), dtype=torch.float64, device=device)
        self.grad = torch.empty(int(tot[1]), dtype=torch.float64, device=device)

    def step(self, backward: bool = True) -> dict:
        N.qs_program_encode(self.ph, self.qs_dtype, self.x, self.states)
        N.qs_program_forward(self.ph, self.qs_dtype, self.params, self.states, self.expz)
        out = {"expz": self.expz, "loss": (self.expz * self.weights).sum()}
        if backward:
            N.qs_program_adjoint(self.ph, self.qs_dtype, self.params, self.states,
                                 self.weights, self.grad)
            out["grad_params"] = self.grad
        return out


class GraphStep:
    """A whole step captured once in a HIP graph (torch.cuda.CUDAGraph) and
    replayed. The first call runs the step eagerly so every plan is built and
    uploaded before the capture; replays reuse the step's device buffers."""

    def __init__(self, fn, warmup: int = 1):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out = fn()

    def replay(self):
        self.graph.replay()
        return self.out
