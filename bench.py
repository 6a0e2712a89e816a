"""Benchmark: forward + adjoint gate-amplitude updates per second.

One step = the whole path over one batch with inputs resident in HBM:
amplitude/angle encoding, forward gate sweep with FP64 Pauli-Z readout, the
loss and dL/d<Z> in torch, and the adjoint backward (FP64 batch-summed
parameter gradients). Work per step = 3 * B * 2^n * G gate-amplitude updates.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

Prints ONE JSON line. Alongside the fused path it times the plain path (one
kernel launch per gate, states in HBM) on the same inputs, the dominant
kernel's duration with HIP events on the launch stream, and the FP64 CPU
oracle on a bounded sample of the batch (the ``cpu_baseline`` leg).
"""

from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adjoint gate-amp updates/s, 10q×4096 batch; % LDS/HBM roofline vs plain"
WORKLOAD_TEXT = {
    "c2": "10 qubits, batch 4096: amplitude-encoded N(0,1) 1024-dim inputs; "
          "8 layers of RX,RY,RZ per qubit + CZ ring (240 params); "
          "MSE(<Z_0>, +-1 labels); complex64 forward + adjoint",
    "c3": "8 qubits, batch 65536: data re-uploading RY(w x + b) x16 layers "
          "+ RZ + CNOT chain; complex64 forward + adjoint (params and inputs)",
    "c4": "12 qubits, batch 1024: 6-layer RY/RZ + CNOT-chain encoder, "
          "decoder its inverse with separate params, 4 trash qubits reset, "
          "loss 1 - fidelity; complex64 forward + adjoint",
    "c1": "4 qubits, batch 64: 2 layers RY,RZ + ring CNOT; complex128 forward",
    "c5b": "26 qubits, one complex64 state (512 MiB in HBM), 20 hardware-efficient "
           "layers (RY,RZ + ring CNOT; 1560 gates), loss sum_q g_q <Z_q>; "
           "forward + adjoint on the tiled large-state path",
}
# MI355X peaks (published): fp32 vector 157.3 TFLOP/s, HBM 8 TB/s.
PEAK_FP32_TFLOPS = 157.3

# Algorithmic flops per amplitude of one gate: a Pauli rotation applied to a
# complex amplitude costs 6 real flops (each output component is two real
# products and one add); the adjoint un-applies it to psi and lam (12) and
# forms Im<lam|P|psi> (4). CNOT, CZ, X, Y, Z, H: counted as 0.
FLOPS_ROT_FWD = 6
FLOPS_ROT_ADJ = 16


# Sources that decide what the adjoint kernel does; the measured HBM traffic
# in profiles/ is only reported while their hash matches the one recorded
# with the counters.
KERNEL_SOURCES = ["paper_2509_25075_amd/csrc/sv_engine.h",
                  "paper_2509_25075_amd/csrc/sv_c64_adj.hip",
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


def measured_traffic(workload: str):
    """HBM bytes per launch of the adjoint kernel from the FETCH_SIZE /
    WRITE_SIZE counters recorded under profiles/ (scaled by a plain copy of
    known size), or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"sv_adjoint_{workload}_traffic.json")
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


def cpu_baseline(key: str, rows: int) -> dict:
    """The FP64 oracle, as it stands, on `rows` rows of the workload, one
    host thread (subprocess with BLAS/OpenMP pinned to 1 thread)."""
    code = f"""
import json, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np
import oracle as O
from workloads import make_workload
w = make_workload({key!r}, {rows})
t0 = time.perf_counter()
feats = w.feats
if w.encoding == "amplitude":
    psi0 = O.encode_amplitude(w.x, w.n_qubits)
else:
    psi0 = O.encode_zero(w.batch, w.n_qubits)
if w.loss == "fidelity_reset":
    psi = O.run_circuit(w.circuit, w.params, None, psi0)
    chi = O.run_circuit(w.decoder, w.params_dec, None, psi0)
    F, c = O.fidelity_reset(psi, chi, w.n_trash)
    dF = -np.ones(w.batch) / w.batch
    lam, mu = O.reset_channel_fidelity_cotangents(psi, chi, c, dF, w.n_trash)
    g1, _ = O.adjoint_vjp(w.circuit, w.params, None, psi0, lam_final=lam)
    g2, _ = O.adjoint_vjp(w.decoder, w.params_dec, None, psi0, lam_final=mu)
else:
    z = O.expz(O.run_circuit(w.circuit, w.params, feats, psi0))
    if w.loss != "none":
        L, dz = O.loss_and_dexpz(w.loss, z, w.labels, w.weights)
        gth, _ = O.adjoint_vjp(w.circuit, w.params, feats, psi0, dexpz=dz)
        O.theta_to_param_grads(w.circuit, w.params, feats, gth)
dt = time.perf_counter() - t0
print(json.dumps({{"seconds": dt, "updates": w.updates_per_step()}}))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
               MKL_NUM_THREADS="1", NUMEXPR_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True,
                         text=True, env=env, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr)
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": r["updates"] / r["seconds"], "unit": "gate-amp updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{rows} rows of the batch, forward + adjoint, "
                      f"{r['seconds']:.1f} s on 1 host thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--cpu-rows", type=int, default=384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the adjoint kernel's sources and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (use the default register split)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB "
                         "(5 launches) and exit: the known-size kernel whose "
                         "FETCH_SIZE / WRITE_SIZE counters scale the engine's")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.copy_calibration:
        import torch
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
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is designed, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_25075_amd import sim
    from workloads import make_workload

    from paper_2509_25075_amd import _native as N

    w = make_workload(args.workload)
    tuned = None
    if not args.no_tune:
        # The library's autotuner times the register-split candidates of each
        # circuit at this batch size; later calls look the choice up.
        tuned = {}
        for name, c in (("circuit", w.circuit), ("decoder", w.decoder)):
            if c is None:
                continue
            s0 = sim.Simulator(c, w.dtype)
            if s0.plan_info(w.batch)["path"] not in (N.QS_PATH_FUSED, N.QS_PATH_HBM):
                continue
            t = N.qs_autotune(s0.h, s0.qs_dtype, w.batch, 0)
            tuned[name] = {k: t[k] for k in ("fwd_log2_regs", "adj_log2_regs",
                                             "tile_qubits")}
        torch.cuda.synchronize()
    d = sim.to_device(w, flags=0)  # automatic: register/LDS engine, else tiled HBM
    path_name = {1: "fused", 2: "plain", 3: "tiled_hbm"}[d.sim.plan_info(w.batch)["path"]]
    updates = w.updates_per_step()
    stream = torch.cuda.current_stream()

    # dominant-kernel events: the adjoint call (one engine launch + a small
    # FP64 reduction of per-block partials) on the launch stream
    adj_events = []
    orig_adjoint = sim.Simulator.adjoint

    def timed_adjoint(self, *a, **k):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r = orig_adjoint(self, *a, **k)
        e1.record(stream)
        adj_events.append((e0, e1))
        return r

    for _ in range(args.warmup):
        sim.step(d)
    torch.cuda.synchronize()
    sim.Simulator.adjoint = timed_adjoint
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        sim.step(d)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sim.Simulator.adjoint = orig_adjoint
    ms = t0.elapsed_time(t1) / args.steps
    value = updates / (ms * 1e-3)
    adj_ms = sum(a.elapsed_time(b) for a, b in adj_events) / max(1, len(adj_events))
    n_adj_per_step = max(1, len(adj_events) // args.steps)

    rot = _rotations(w.circuit) + (_rotations(w.decoder) if w.decoder else 0)
    flops_adj = FLOPS_ROT_ADJ * (rot // (2 if w.decoder else 1)) * (1 << w.n_qubits) * w.batch
    achieved = flops_adj / (adj_ms * 1e-3) / 1e12 if w.loss != "none" else None

    plain = None
    if not args.no_plain and w.loss != "none":
        dp = sim.to_device(w, flags=2)
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

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, min(args.cpu_rows, w.batch))

    rec = {
        "metric": METRIC, "value": value, "unit": "gate-amp updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32" if w.dtype == "c64" else "fp64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}",
                   "batch": w.batch, "qubits": w.n_qubits,
                   "gates": w.circuit.n_gates + (w.decoder.n_gates if w.decoder else 0),
                   "updates_per_step": updates, "path": path_name, "tuned": tuned},
        "roofline": None if achieved is None else {
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic(args.workload), "kernel": "sv_adjoint",
            "kernel_ms": adj_ms / 1.0, "launches_per_step": n_adj_per_step,
            "algorithmic_flops_per_launch": flops_adj},
        "cpu_baseline": cpu,
        "plain": plain,
        "speedup_vs_plain": None if plain is None else value / plain["value"],
        "wall_s": wall,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
