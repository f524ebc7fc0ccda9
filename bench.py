#!/usr/bin/env python3
"""Throughput of the tensor-network contraction path on one MI355X.

Default workload (--config 1): the 24-qubit random brickwork circuit of depth
16 (U3 layers and alternating CZ pairs, seeded), with one-qubit gates
pre-contracted into the two-qubit blocks, contracted along the searched order
into the full 2^24 complex64 statevector.  One step = one whole pass of the
path: gate materialisation from the angles on the device, every pairwise
contraction, and the result in qubit order.  Inputs are resident on the GPU
before the timed region; the plan is made once, outside it (its time is
reported).

Other workloads (--config): 0 = 10-qubit brickwork statevector, 2 = 4096
amplitudes of the 32-qubit 4x8 grid circuit, 3 = <C> of 512 batched QAOA
MaxCut circuits, 4 = adjoint gradients of a 20-qubit ansatz for 64 parameter
vectors.

Prints one JSON line: the metric, value, the dominant kernel's roofline
fraction measured with HIP events during the timed region, and the FP64 CPU
oracle timed on the host as a baseline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TN contraction TFLOP/s (% MFMA peak), amplitudes/s, grads/s at ≤1e-5 vs FP64"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0


def relerr(got, want):
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    want = np.asarray(want, dtype=np.complex128).reshape(-1)
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


class Workload:
    """setup() builds everything, step() runs one pass, result() returns the
    output for the check, units_per_step is the metric's unit count."""

    def check(self):
        return None

    def cpu_baseline(self):
        return None


class Statevector(Workload):
    def __init__(self, tnq, torch, circ, name, fuse, kind, trials, precision):
        self.tnq, self.torch, self.circ, self.name, self.precision = tnq, torch, circ, name, precision
        t0 = time.perf_counter()
        self.net = tnq.Network.from_circuit(circ, fuse=fuse)
        self.path = self.net.plan(kind, trials=trials)
        self.plan_s = time.perf_counter() - t0
        n = circ.n_qubits
        self.out = torch.empty(1, 1 << n, dtype=torch.complex64, device="cuda")
        self.ws = torch.empty(self.path.workspace_bytes(1), dtype=torch.uint8, device="cuda")
        self.unit, self.units_per_step = "amplitudes/s", float(1 << n)
        self.config = {"workload": name, "n_qubits": n, "path": kind, "fuse": fuse, "precision": precision}

    def step(self):
        self.tnq.contract_path(self.net, self.path, precision=self.precision, out=self.out, workspace=self.ws)

    def tune(self):
        return self.tnq.autotune(self.net, self.path, precision=self.precision, workspace=self.ws)

    def check(self):
        import oracle
        t0 = time.perf_counter()
        self.psi_ref = oracle.statevector(self.circ)
        self.cpu_s = time.perf_counter() - t0
        return relerr(self.out[0].cpu().numpy(), self.psi_ref)

    def cpu_baseline(self):
        import oracle
        return {"value": self.units_per_step / self.cpu_s, "unit": self.unit, "cores": oracle.num_threads(),
                "kind": "oracle", "sample": f"one full statevector of the same circuit (FP64 gate-by-gate, "
                                            f"{len(self.circ.gates)} gates), {self.cpu_s:.2f} s"}


class Amplitudes(Workload):
    def __init__(self, tnq, torch, trials, precision):
        import workloads
        self.tnq, self.torch, self.precision = tnq, torch, precision
        self.circ, bits = workloads.config2()
        t0 = time.perf_counter()
        self.net = tnq.Network.from_circuit(self.circ, output="amplitudes", n_bitstrings=len(bits))
        self.path = self.net.plan("search", max_log2_intermediate=28, trials=trials)
        self.plan_s = time.perf_counter() - t0
        self.bits = torch.as_tensor(bits.view(np.int64), device="cuda")
        self.out = torch.empty(len(bits), dtype=torch.complex64, device="cuda")
        self.ws = torch.empty(self.path.workspace_bytes(1), dtype=torch.uint8, device="cuda")
        self.unit, self.units_per_step = "amplitudes/s", float(len(bits))
        self.config = {"workload": "32-qubit 4x8 grid circuit, depth 12, 4096 seeded bitstrings on a batch index",
                       "n_qubits": 32, "n_bitstrings": len(bits), "path": "search", "precision": precision}

    def step(self):
        self.tnq.amplitudes(self.net, self.path, self.bits, precision=self.precision, out=self.out, workspace=self.ws)

    def tune(self):
        return self.tnq.autotune(self.net, self.path, precision=self.precision, workspace=self.ws)


class QAOA(Workload):
    def __init__(self, tnq, torch, precision):
        import workloads
        self.tnq, self.torch, self.precision = tnq, torch, precision
        self.inst = workloads.config3()
        t0 = time.perf_counter()
        self.nets = [tnq.Network.from_circuit(it.circuit) for it in self.inst]
        self.paths = [nt.plan("sequential") for nt in self.nets]
        self.plan_s = time.perf_counter() - t0
        self.obs = [tnq.Observable(*workloads.maxcut_observable(it.circuit.n_qubits, it.edges)) for it in self.inst]
        self.params = [torch.as_tensor(it.params, device="cuda").reshape(1, -1) for it in self.inst]
        self.unit, self.units_per_step = "expectations/s", float(len(self.inst))
        self.config = {"workload": "512 QAOA MaxCut circuits, n in {16..26}, 3-regular graphs, p=4, <C> in FP64",
                       "n_circuits": len(self.inst), "path": "sequential", "precision": precision}
        self.ws = None

    def step(self):
        self.out = self.tnq.expectation(self.nets, self.paths, self.params, self.obs, precision=self.precision,
                                        workspace=self.ws)

    def cpu_baseline(self):
        import oracle
        import workloads
        t0 = time.perf_counter()
        k = 0
        for it in self.inst:
            if time.perf_counter() - t0 > 15.0:
                break
            m, c = workloads.maxcut_observable(it.circuit.n_qubits, it.edges)
            oracle.circuit_expectation(it.circuit, it.params, m, c)
            k += 1
        dt = time.perf_counter() - t0
        return {"value": k / dt, "unit": self.unit, "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"the first {k} of the 512 circuits ({dt:.1f} s)"}


class Gradients(Workload):
    def __init__(self, tnq, torch, precision):
        import workloads
        self.tnq, self.torch, self.precision = tnq, torch, precision
        self.circ, params, (m, c) = workloads.config4()
        self.m, self.c, self.params_np = m, c, params
        t0 = time.perf_counter()
        self.net = tnq.Network.from_circuit(self.circ)
        self.path = self.net.plan("sequential")
        self.plan_s = time.perf_counter() - t0
        self.obs = tnq.Observable(m, c)
        self.params = torch.as_tensor(params, device="cuda")
        self.batch = params.shape[0]
        self.ws = torch.empty(int(tnq.lib().tn_backward_workspace_bytes(self.net.handle, self.path.handle,
                                                                         self.batch)), dtype=torch.uint8,
                              device="cuda")
        self.unit, self.units_per_step = "grads/s", float(self.batch * self.circ.n_params)
        self.config = {"workload": "20-qubit hardware-efficient ansatz, 10 layers, 400 angles, 64 parameter "
                                   "vectors, loss sum_i <Z_i Z_i+1>, adjoint gradient",
                       "n_qubits": 20, "batch": self.batch, "n_params": self.circ.n_params, "path": "sequential",
                       "precision": precision}

    def tune(self):
        return self.tnq.autotune(self.net, self.path, self.params, batch=self.batch, precision=self.precision,
                                 workspace=self.ws)

    def step(self):
        self.value, self.grad = self.tnq.backward(self.net, self.path, self.params, self.obs, batch=self.batch,
                                                  precision=self.precision, workspace=self.ws)

    def cpu_baseline(self):
        import oracle
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 15.0 and k < self.circ.n_params:
            oracle.param_shift_gradient(self.circ, self.params_np[0], self.m, self.c, which=[k])
            k += 1
        dt = time.perf_counter() - t0
        return {"value": k / dt, "unit": self.unit, "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"exact parameter-shift derivatives of the first {k} angles of vector 0 ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=1, choices=[0, 1, 2, 3, 4])
    ap.add_argument("--path", default="search", help="search | greedy | sequential | random (configs 0, 1)")
    ap.add_argument("--trials", type=int, default=128, help="randomised orders tried by the search")
    ap.add_argument("--fuse", default="split", help="split | dense | none (configs 0, 1)")
    ap.add_argument("--precision", default="c64", help="c64 | bf16x3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the parity check against the oracle")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes (no autotuning)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_2108_06831_amd as tnq

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    fuse = False if args.fuse == "none" else args.fuse
    if args.config == 1:
        wl = Statevector(tnq, torch, workloads.config1(),
                         "24-qubit random brickwork circuit, depth 16 (384 U3 + 184 CZ, seeded), 2-qubit fusion, "
                         "full 2^24 complex64 statevector", fuse, args.path, args.trials, args.precision)
    elif args.config == 0:
        wl = Statevector(tnq, torch, workloads.config0(),
                         "10-qubit random brickwork circuit, depth 8, full 2^10 complex64 statevector", fuse,
                         args.path, args.trials, args.precision)
    elif args.config == 2:
        wl = Amplitudes(tnq, torch, args.trials, args.precision)
    elif args.config == 3:
        wl = QAOA(tnq, torch, args.precision)
    else:
        wl = Gradients(tnq, torch, args.precision)

    tune = None
    if not args.no_tune and hasattr(wl, "tune"):
        t0 = time.perf_counter()
        tune = wl.tune()
        tune["tune_seconds"] = time.perf_counter() - t0
    for _ in range(args.warmup):
        wl.step()
    torch.cuda.synchronize()
    print(f"[bench] config {args.config}: warmup done ({args.warmup} steps), timing {args.steps} steps",
          file=sys.stderr, flush=True)

    tnq.profile_reset()
    tnq.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        wl.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tnq.profile_enable(False)
    prof = tnq.profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    value = wl.units_per_step / (ms * 1e-3)

    # dominant kernel by measured time
    kind, rec = max(prof.items(), key=lambda kv: kv[1]["seconds"])
    if kind == "gemm":
        # BF16x3 needs three bf16 products per product term: its ceiling is a third of the bf16 peak
        peak = PEAK_FP32_MFMA_TFLOPS if args.precision == "c64" else PEAK_BF16_MFMA_TFLOPS / 3
        achieved = rec["flops"] / rec["seconds"] / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None}
    else:
        achieved = rec["bytes"] / rec["seconds"] / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof.update({"kernel": kind, "launches_per_step": rec["launches"] / args.steps,
                 "avg_launch_us": rec["seconds"] / rec["launches"] * 1e6})
    kernels = {k: {"launches_per_step": v["launches"] / args.steps, "ms_per_step": v["seconds"] * 1e3 / args.steps,
                   "GB/s": v["bytes"] / max(v["seconds"], 1e-30) / 1e9,
                   "TFLOP/s": v["flops"] / max(v["seconds"], 1e-30) / 1e12} for k, v in prof.items()}
    config = dict(wl.config)
    config["plan_seconds"] = wl.plan_s
    if tune is not None:
        config["autotune"] = tune
    if hasattr(wl, "path"):
        st = wl.path.stats
        config.update({"path_flops": st["flops"], "path_bytes": st["bytes"],
                       "max_intermediate": st["max_intermediate_elems"], "n_steps": st["n_steps"],
                       "n_small_steps": st["n_small_steps"], "modeled_ms": st["modeled_seconds"] * 1e3})
    result = {
        "metric": METRIC,
        "value": value,
        "unit": wl.unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if args.precision == "c64" else "c64-bf16x3",
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "kernels": kernels,
    }
    if hasattr(wl, "path"):
        result["path_tflops"] = wl.path.stats["flops"] / (ms * 1e-3) / 1e12
    if not args.no_check:
        err = wl.check()
        if err is not None:
            result["rel_err_vs_oracle"] = err
    if not args.no_cpu_baseline:
        if args.no_check and isinstance(wl, Statevector):
            wl.check()
        cb = wl.cpu_baseline()
        if cb is not None:
            result["cpu_baseline"] = cb
    print(json.dumps(result))


if __name__ == "__main__":
    main()
