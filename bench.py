"""Benchmark: forward + adjoint gate-amplitude updates per second.

One step = the whole path over one batch with inputs resident in HBM:
amplitude/angle encoding, forward gate sweep with FP64 Pauli-Z (or fidelity)
readout, the loss and its upstream gradient in torch, and the adjoint
backward (FP64 batch-summed parameter gradients). Work per step =
3 * B * 2^n * G gate-amplitude updates (forward sweep, then uncompute and
propagate in the backward).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

Prints ONE JSON line. The default workload is the 10-qubit x 4096 batch
(c2). Alongside the fused path it times the plain path (one kernel launch per
gate, states in HBM) on the same inputs, the dominant kernel's duration with
HIP events on the launch stream, and the FP64 CPU oracle on a bounded sample
of the batch (the ``cpu_baseline`` leg, c2 only).
"""

from __future__ import annotations

import argparse
import dataclasses
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adjoint gate-amp updates/s, 10q×4096 batch; % LDS/HBM roofline vs plain"
WORKLOAD_TEXT = {
    "c1": "4 qubits, batch 64: 2 layers RY,RZ + ring CNOT; complex128 forward",
    "c2": "10 qubits, batch 4096: amplitude-encoded N(0,1) 1024-dim inputs; "
          "8 layers of RX,RY,RZ per qubit + CZ ring (240 params); "
          "MSE(<Z_0>, +-1 labels); complex64 forward + adjoint",
    "c3": "8 qubits, batch 65536: data re-uploading RY(w x + b) x16 layers "
          "+ RZ + CNOT chain; complex64 forward + adjoint (params and inputs)",
    "c4": "12 qubits, batch 1024: 6-layer RY/RZ + CNOT-chain encoder, "
          "decoder its inverse with separate params, 4 trash qubits reset, "
          "loss 1 - fidelity; complex64 forward + adjoint",
    "c5a": "10000 independent circuits, n ~ U{6..14}, depth ~ U{4..32} "
           "hardware-efficient layers (RY,RZ + ring CNOT), one amplitude-encoded "
           "N(0,1) input each, loss sum_q g_q <Z_q>; one persistent launch per "
           "direction; complex64 forward + adjoint",
    "c5b": "26 qubits, one complex64 state (512 MiB in HBM; 1 GiB in complex128), 20 hardware-efficient "
           "layers (RY,RZ + ring CNOT; 1560 gates), loss sum_q g_q <Z_q>, state "
           "checkpoints every 4 layers; forward + adjoint on the tiled large-state "
           "path",
}


def workload_text(key, dtype, loss=None):
    t = WORKLOAD_TEXT[key]
    if loss == "fidelity_postselect":
        t = t.replace("4 trash qubits reset, loss 1 - fidelity",
                      "4 trash qubits measured with only the all-zero outcome kept "
                      "(renormalised in FP64), loss 1 - post-selected fidelity")
    elif loss == "fidelity_trajectory":
        t = t.replace("4 trash qubits reset, loss 1 - fidelity",
                      "4 trash qubits reset along one sampled trajectory per sample "
                      "(measurement outcome drawn from seeded uniforms), loss 1 - "
                      "trajectory fidelity")
    return t.replace("complex64 forward", "complex128 forward") if dtype == "c128" else t


# MI355X published peaks: fp32 vector 157.3 TFLOP/s, HBM 8 TB/s.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
# Issue-rate ceiling of unpacked FP32 FMAs (no v_pk_* instructions in this
# library): 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz. The published
# 157.3 counts packed (two-wide) FP32; FP64 FMAs issue at this same rate.
ISSUE_FP32_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0
# LDS: 128 B per clock per CU (the CDNA figure; not re-measured here) x 256
# CUs x 2.4 GHz. Used only for the pass-equivalent context figure.
LDS_TBPS_ASSUMED = 78.6

# Algorithmic flops per amplitude of one gate: a Pauli rotation applied to a
# complex amplitude costs 6 real flops (each output component is two real
# products and one add); the adjoint un-applies it to psi and lam (12) and
# forms Im<lam|P|psi> (4). CNOT, CZ, X, Y, Z, H: counted as 0.
FLOPS_ROT_FWD = 6
FLOPS_ROT_ADJ = 16
# ... and of one rotation on one amplitude in the forward sweep (two products
# and one add per output component).
FLOPS_ROT_FWD = 6

# Sources that decide what the adjoint kernel does; the measured HBM traffic
# in profiles/ is only reported while their hash matches the one recorded
# with the counters.
KERNEL_SOURCES = ["paper_2509_25075_amd/csrc/sv_engine.h",
                  "paper_2509_25075_amd/csrc/sv_c64_adj.hip",
                  "paper_2509_25075_amd/csrc/sv_c64_train.hip",
                  "paper_2509_25075_amd/csrc/qs_internal.h",
                  "paper_2509_25075_amd/csrc/planner.cpp",
                  "include/qs.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str = "sv_adjoint"):
    """HBM bytes per launch of the dominant kernel from the FETCH_SIZE /
    WRITE_SIZE counters recorded under profiles/ (scaled by a plain copy of
    known size), or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != kernel_source_hash():
        return None
    return d["bytes_per_launch"]


def _rotations(circuit):
    import numpy as np
    return int(np.isin(circuit.gates["op"], (0, 1, 2)).sum())


# ------------------------------------------------------------ CPU baseline
_CPU_WORKER = """
import json, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import oracle as O
from workloads import make_workload
w = make_workload({key!r}, {rows})
if {gates}:  # one state too large to split: the first gates of the circuit on all of it
    from workloads import circuits as C
    w = w.__class__(**{{**w.__dict__, "circuit": C.Circuit(w.n_qubits, w.circuit.gates[:{gates}],
                                                        w.circuit.n_params)}})
k, W = {part}, {parts}
sl = slice(k, None, W)
x = w.x[sl] if w.x is not None else None
feats = w.feats[sl] if w.feats is not None else None
labels = w.labels[sl] if w.labels is not None else None
B = len(range(*sl.indices(w.batch)))
t0 = time.perf_counter()
if w.encoding == "amplitude":
    psi0 = O.encode_amplitude(x, w.n_qubits)
else:
    psi0 = O.encode_zero(B, w.n_qubits)
if w.loss == "fidelity_reset":
    psi = O.run_circuit(w.circuit, w.params, None, psi0)
    chi = O.run_circuit(w.decoder, w.params_dec, None, psi0)
    F, c = O.fidelity_reset(psi, chi, w.n_trash)
    dF = -np.ones(B) / B
    lam, mu = O.reset_channel_fidelity_cotangents(psi, chi, c, dF, w.n_trash)
    O.adjoint_vjp(w.circuit, w.params, None, psi0, lam_final=lam)
    O.adjoint_vjp(w.decoder, w.params_dec, None, psi0, lam_final=mu)
else:
    z = O.expz(O.run_circuit(w.circuit, w.params, feats, psi0))
    if w.loss != "none":
        L, dz = O.loss_and_dexpz(w.loss, z, labels, w.weights)
        gth, _ = O.adjoint_vjp(w.circuit, w.params, feats, psi0, dexpz=dz)
        O.theta_to_param_grads(w.circuit, w.params, feats, gth)
dt = time.perf_counter() - t0
G = w.circuit.n_gates + (w.decoder.n_gates if w.decoder else 0)
passes = 1 if w.loss == "none" else 3
print(json.dumps({{"seconds": dt, "updates": passes * B * (1 << w.n_qubits) * G}}))
"""


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The CPU share of one GPU on the GPU hosts these benchmarks run on is 16
# cores; the oracle's worker processes stay within it.
CPU_SHARE = 16


def cpu_baseline(key: str, rows_per_worker: int, gates: int = 0) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    one process per available host core (at most the 16-core share of one
    GPU), each with one BLAS/OpenMP thread, each on its own rows of the
    sample. With ``gates`` > 0 (a single state too large to split), one
    process runs the first ``gates`` gates of the circuit on the whole state,
    forward with readout and adjoint."""
    avail = len(os.sched_getaffinity(0))
    workers = 1 if gates else max(1, min(CPU_SHARE, avail))
    rows = rows_per_worker * workers
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
               MKL_NUM_THREADS="1", NUMEXPR_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, "-c", _CPU_WORKER.format(
        root=ROOT, key=key, rows=None if gates else rows, part=k, parts=workers,
        gates=gates)],
        stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
        for k in range(workers)]
    res = []
    for p in procs:
        out, err = p.communicate(timeout=900)
        if p.returncode != 0:
            raise RuntimeError(err)
        res.append(json.loads(out.strip().splitlines()[-1]))
    wall = max(r["seconds"] for r in res)
    updates = sum(r["updates"] for r in res)
    sample = (f"the first {gates} gates of the circuit on the whole state (forward with "
              f"readout, loss and adjoint; 1 process x 1 thread), {wall:.1f} s wall"
              if gates else
              f"{rows} rows of the batch ({rows_per_worker} per process, {workers} "
              f"processes x 1 thread), forward + adjoint, {wall:.1f} s wall")
    return {"value": updates / wall, "unit": "gate-amp updates/s",
            "cores": workers, "kind": "oracle", "sample": sample,
            "host": {"cpu_model": cpu_model(), "cores_visible": avail,
                     "cores_online": os.cpu_count(), "process_cap": CPU_SHARE}}


# ---------------------------------------------------------------- timing
class AdjointTimer:
    """HIP events around every call of the dominant library call (the
    adjoint) on the launch stream during the timed region."""

    def __init__(self, torch, stream):
        self.torch, self.stream, self.ev, self.on = torch, stream, [], False
        self.extra_warmup = 0  # untimed steps run after the W warm-up steps

    def wrap(self, fn):
        def timed(*a, **k):
            if not self.on:
                return fn(*a, **k)
            e0 = self.torch.cuda.Event(enable_timing=True)
            e1 = self.torch.cuda.Event(enable_timing=True)
            e0.record(self.stream)
            r = fn(*a, **k)
            e1.record(self.stream)
            self.ev.append((e0, e1))
            return r
        return timed

    def mean_ms(self):
        return sum(a.elapsed_time(b) for a, b in self.ev) / max(1, len(self.ev))


# Untimed warm-up runs at least this long (after the W warm-up steps, more
# untimed steps until it is reached): the GPU raises its clocks over the
# first few milliseconds of sustained work, and a short timed region that
# starts before that measures the ramp rather than the step.
WARMUP_MIN_S = 0.3


def timed_loop(torch, stream, step, steps, warmup, timer):
    w0 = time.perf_counter()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    timer.extra_warmup = 0
    while time.perf_counter() - w0 < WARMUP_MIN_S:
        for _ in range(4):
            step()
        torch.cuda.synchronize()
        timer.extra_warmup += 4
    timer.on = True
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    wall0 = time.perf_counter()
    for _ in range(steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    timer.on = False
    return t0.elapsed_time(t1) / steps, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--dtype", choices=["c64", "c128"], default=None,
                    help="run the workload in this complex type (default: its own)")
    ap.add_argument("--fidelity", choices=["reset", "postselect", "trajectory"],
                    default="reset",
                    help="c4: trash qubits reset (default), measured with only "
                         "the all-zero outcome kept and renormalised, or reset "
                         "along one sampled trajectory per sample")
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--cpu-rows", type=int, default=256,
                    help="oracle rows per host process for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB "
                         "(5 launches) and exit: the known-size kernel whose "
                         "FETCH_SIZE / WRITE_SIZE counters scale the engine's")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the adjoint kernel's sources and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (use the default register split)")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is designed, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_25075_amd import sim
    from paper_2509_25075_amd import _native as N
    from workloads import make_workload, uneven_batch
    from workloads.data import trajectory_uniforms

    if args.copy_calibration:
        n = args.copy_calibration << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": args.copy_calibration,
                          "bytes_read_per_launch": 4 * n,
                          "bytes_written_per_launch": 4 * n}))
        return

    stream = torch.cuda.current_stream()
    timer = AdjointTimer(torch, stream)
    key = args.workload
    plain = None
    extra = {}

    if key == "c5a":
        ub = uneven_batch()
        dev = sim.UnevenDevice(ub, dtype=args.dtype or "c64")
        updates = ub.updates_per_step()
        N.qs_program_adjoint = timer.wrap(N.qs_program_adjoint)
        ms, wall = timed_loop(torch, stream, dev.step, args.steps, args.warmup, timer)
        rot_amp = sum(len(idx) * (1 << n) * _rotations(c) for n, _, c, idx in ub.classes)
        flops_adj = FLOPS_ROT_ADJ * rot_amp
        adj_ms = timer.mean_ms()
        roof = {"bound": "alu", "achieved": flops_adj / (adj_ms * 1e-3) / 1e12,
                "peak": PEAK_FP64_TFLOPS if args.dtype == "c128" else PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "traffic": None,
                "kernel": "sv_program (adjoint)" if dev.dtype == "c64" else
                "qs_program_adjoint (sv_program; 14-qubit classes on the tiled path)",
                "kernel_ms": adj_ms,
                "launches_per_step": 1, "algorithmic_flops_per_launch": flops_adj}
        roof["frac"] = roof["achieved"] / roof["peak"]
        if args.dtype != "c128":
            roof["unpacked_fp32_ceiling"] = ISSUE_FP32_TFLOPS
            roof["frac_of_unpacked_ceiling"] = roof["achieved"] / ISSUE_FP32_TFLOPS
        cfg = {"workload": f"c5a: {workload_text(key, args.dtype)}", "circuits": ub.n_circuits,
               "classes": len(ub.classes), "updates_per_step": updates,
               "path": "persistent", "complex": args.dtype or "c64"}
        dtype = "fp64" if args.dtype == "c128" else "fp32"
    else:
        w = make_workload(key)
        if args.dtype:
            w = dataclasses.replace(w, dtype=args.dtype)
        if key == "c4" and args.fidelity != "reset":
            w = dataclasses.replace(w, loss="fidelity_" + args.fidelity)
        traj_u = trajectory_uniforms(w.batch) if w.loss == "fidelity_trajectory" else None
        tuned = None
        if not args.no_tune:
            # The library's autotuner times the register-split candidates of
            # each circuit at this batch size; later calls look the choice up.
            tuned = {}
            for name, c in (("circuit", w.circuit), ("decoder", w.decoder)):
                if c is None:
                    continue
                s0 = sim.Simulator(c, w.dtype)
                if s0.plan_info(w.batch)["path"] not in (N.QS_PATH_FUSED, N.QS_PATH_HBM,
                                                         N.QS_PATH_MFMA):
                    continue
                t = N.qs_autotune(s0.h, s0.qs_dtype, w.batch, 0)
                tuned[name] = {k: t[k] for k in ("path", "fwd_log2_regs", "adj_log2_regs",
                                                 "tile_qubits", "fwd_samples_cap",
                                                 "adj_samples_cap", "fwd_half_staging",
                                                 "adj_half_staging", "fwd_ms", "adj_ms")}
            torch.cuda.synchronize()
        ck = 4 if key == "c5b" else 0
        # automatic path: register/LDS engine when it fits, else tiled HBM
        d = sim.to_device(w, flags=0, ckpt_every_layers=ck, traj_u=traj_u)
        path = {1: "fused", 2: "plain", 3: "tiled_hbm", 4: "mfma_blocks"}[
            d.sim.plan_info(w.batch)["path"]]
        updates = w.updates_per_step()
        # The dominant call: the one-launch training step where it runs,
        # else the adjoint.
        one_launch = w.loss != "none" and sim.train_step_runs(d)
        if one_launch:
            N.qs_train_step_mse = timer.wrap(N.qs_train_step_mse)
        else:
            sim.Simulator.adjoint = timer.wrap(sim.Simulator.adjoint)
        ms, wall = timed_loop(torch, stream, lambda: sim.step(d), args.steps,
                              args.warmup, timer)
        adj_ms = timer.mean_ms()
        n_adj = max(1, len(timer.ev) // args.steps)
        rot = _rotations(w.circuit)
        amps = (1 << w.n_qubits) * w.batch
        if w.loss == "none":
            roof = None
        elif path == "tiled_hbm":
            # Each epoch's adjoint launch reads psi and lam and writes them
            # back (4 complex amplitudes of 8 or 16 B); the timed call runs
            # all epochs of the plan with the step's checkpoints, plus its own
            # state copies: psi_G into the workspace (read + write), lam
            # formed from it (read + write) and one re-anchoring copy per
            # checkpoint (read + write).
            hi = N.qs_hbm_info_get(d.sim.h, d.sim.qs_dtype, w.batch, 0, d.ckpt_gates)
            n_ep = hi["n_passes"]
            cs = 8 if w.dtype == "c64" else 16
            n_ck = len(d.ckpt_gates or [])
            bytes_call = (n_ep * 4 + 4 + 2 * n_ck) * cs * amps
            roof = {"bound": "hbm", "achieved": bytes_call / (adj_ms * 1e-3) / 1e9,
                    "peak": PEAK_HBM_GBPS, "unit": "GB/s", "traffic": None,
                    "kernel": "sv_adjoint (tiled epochs)", "kernel_ms": adj_ms,
                    "launches_per_step": n_ep, "algorithmic_bytes_per_call": bytes_call}
        elif path == "mfma_blocks":
            # Each block's adjoint pass reads psi and lam and writes them back
            # (32 B per complex64 amplitude) and does 768 MFMA flops per
            # amplitude: M^dagger applied to psi and to lam (256 each, the real
            # embedding of a 32 x 32 complex matrix) and rho = sum psi lam^dagger
            # (256); plus the call's state copies as on the tiled path.
            hi = N.qs_hbm_info_get(d.sim.h, d.sim.qs_dtype, w.batch, 0, d.ckpt_gates)
            n_bl = hi["n_passes"]
            n_ck = len(d.ckpt_gates or [])
            bytes_call = (n_bl * 4 + 4 + 2 * n_ck) * 8 * amps
            mfma_flops = n_bl * 768 * amps
            roof = {"bound": "hbm", "achieved": bytes_call / (adj_ms * 1e-3) / 1e9,
                    "peak": PEAK_HBM_GBPS, "unit": "GB/s", "traffic": None,
                    "kernel": "db_adjoint (dense 5-qubit blocks on MFMA)", "kernel_ms": adj_ms,
                    "launches_per_step": n_bl, "algorithmic_bytes_per_call": bytes_call,
                    "mfma_tflops": mfma_flops / (adj_ms * 1e-3) / 1e12,
                    "mfma_frac": mfma_flops / (adj_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
        elif one_launch:
            # forward, readout, loss and adjoint in one launch (plus the
            # partial-sum reduction in the same library call)
            flops_step = (FLOPS_ROT_FWD + FLOPS_ROT_ADJ) * rot * amps
            roof = {"bound": "alu", "achieved": flops_step / (adj_ms * 1e-3) / 1e12,
                    "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                    "traffic": measured_traffic(key, "sv_train"),
                    "kernel": "sv_train (forward, loss and adjoint in one launch)",
                    "kernel_ms": adj_ms, "launches_per_step": n_adj,
                    "algorithmic_flops_per_launch": flops_step}
        else:
            flops_adj = FLOPS_ROT_ADJ * rot * amps
            roof = {"bound": "alu", "achieved": flops_adj / (adj_ms * 1e-3) / 1e12,
                    "peak": PEAK_FP32_TFLOPS if w.dtype == "c64" else PEAK_FP64_TFLOPS,
                    "unit": "TFLOP/s",
                    "traffic": measured_traffic(key) if w.dtype == "c64" else None,
                    "kernel": "sv_adjoint",
                    "kernel_ms": adj_ms, "launches_per_step": n_adj,
                    "algorithmic_flops_per_launch": flops_adj}
        if roof is not None:
            roof["frac"] = roof["achieved"] / roof["peak"]
            if roof["bound"] == "alu" and w.dtype == "c64":
                roof["unpacked_fp32_ceiling"] = ISSUE_FP32_TFLOPS
                roof["frac_of_unpacked_ceiling"] = roof["achieved"] / ISSUE_FP32_TFLOPS
        if not args.no_plain and w.loss != "none" and path == "fused":
            dp = sim.to_device(w, flags=N.QS_PATH_PLAIN, traj_u=traj_u)
            sim.step(dp)
            torch.cuda.synchronize()
            p0 = torch.cuda.Event(enable_timing=True)
            p1 = torch.cuda.Event(enable_timing=True)
            p0.record(stream)
            for _ in range(args.plain_steps):
                sim.step(dp)
            p1.record(stream)
            torch.cuda.synchronize()
            pms = p0.elapsed_time(p1) / args.plain_steps
            plain = {"value": updates / (pms * 1e-3), "ms_per_step": pms}
            del dp
        cfg = {"workload": f"{key}: {workload_text(key, w.dtype, w.loss)}", "complex": w.dtype,
               "batch": w.batch,
               "qubits": w.n_qubits,
               "gates": w.circuit.n_gates + (w.decoder.n_gates if w.decoder else 0),
               "updates_per_step": updates, "path": path, "tuned": tuned}
        if d.ckpt_gates:
            cfg["checkpoints_after_gates"] = d.ckpt_gates
        dtype = "fp32" if w.dtype == "c64" else "fp64"
        if path == "fused":
            # context: updates/s x 16 B (one LDS round trip per gate-amplitude
            # in complex64) over the LDS peak; above 1 means gates applied from
            # registers without an LDS pass each.
            extra["pass_equivalent_lds_frac"] = (updates / (ms * 1e-3)) * 16 / (
                LDS_TBPS_ASSUMED * 1e12)

    value = updates / (ms * 1e-3)
    cpu = None
    if not args.no_cpu_baseline and key == "c2":
        cpu = cpu_baseline(key, args.cpu_rows)
    elif not args.no_cpu_baseline and key == "c5b":
        cpu = cpu_baseline(key, 1, gates=2)
    rec = {
        "metric": METRIC, "value": value, "unit": "gate-amp updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "warmup_extra_steps": timer.extra_warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": cfg, "roofline": roof, "cpu_baseline": cpu, "plain": plain,
        "speedup_vs_plain": None if plain is None else value / plain["value"],
        "wall_s": wall, **extra,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
