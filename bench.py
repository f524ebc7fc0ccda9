#!/usr/bin/env python3
"""Throughput of the tensor-network contraction path on one MI355X.

Workload: the 24-qubit random brickwork circuit of depth 16 (U3 layers and
alternating CZ pairs, seeded), with one-qubit gates pre-contracted into the
two-qubit blocks, contracted along the planned order into the full 2^24
complex64 statevector.  One step = one whole pass of the path: gate
materialisation from the angles on the device, every pairwise contraction,
and the final layout into qubit order.  Inputs are resident on the GPU before
the timed region; the plan is made once, outside it.

Prints one JSON line (metric, value in amplitudes/s, the dominant kernel's
roofline fraction measured with HIP events during the timed region, and the
FP64 CPU oracle timed on the host as a baseline).
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--path", default="search", help="search | greedy | sequential | random")
    ap.add_argument("--trials", type=int, default=128, help="randomised orders tried by the search")
    ap.add_argument("--fuse", default="split", help="split | dense | none")
    ap.add_argument("--precision", default="c64", help="c64 | bf16x3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the parity check against the oracle")
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
    dev = torch.device("cuda:0")
    circ = workloads.config1()
    n = circ.n_qubits
    t0 = time.perf_counter()
    net = tnq.Network.from_circuit(circ, fuse=False if args.fuse == "none" else args.fuse)
    path = net.plan(args.path, trials=args.trials)
    plan_s = time.perf_counter() - t0
    out = torch.empty(1, 1 << n, dtype=torch.complex64, device=dev)
    ws = torch.empty(path.workspace_bytes(1), dtype=torch.uint8, device=dev)

    def step():
        tnq.contract_path(net, path, precision=args.precision, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps), timing {args.steps} steps", file=sys.stderr, flush=True)

    tnq.profile_reset()
    tnq.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tnq.profile_enable(False)
    prof = tnq.profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    value = (1 << n) / (ms * 1e-3)

    # dominant kernel by measured time
    kind, rec = max(prof.items(), key=lambda kv: kv[1]["seconds"])
    per_launch_s = rec["seconds"] / rec["launches"]
    if kind == "gemm":
        achieved = rec["flops"] / rec["seconds"] / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_MFMA_TFLOPS, "traffic": None}
    else:
        achieved = rec["bytes"] / rec["seconds"] / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof.update({"kernel": kind, "launches_per_step": rec["launches"] / args.steps,
                 "avg_launch_us": per_launch_s * 1e6})
    kernels = {k: {"launches_per_step": v["launches"] / args.steps, "ms_per_step": v["seconds"] * 1e3 / args.steps,
                   "GB/s": v["bytes"] / max(v["seconds"], 1e-30) / 1e9,
                   "TFLOP/s": v["flops"] / max(v["seconds"], 1e-30) / 1e12} for k, v in prof.items()}

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if args.precision == "c64" else "c64-bf16x3",
        "data": "synthetic",
        "config": {"workload": "24-qubit random brickwork circuit, depth 16 (384 U3 + 184 CZ, seeded), "
                               "2-qubit fusion, full 2^24 complex64 statevector",
                   "n_qubits": n, "depth": 16, "path": args.path, "fuse": args.fuse, "precision": args.precision,
                   "plan_seconds": plan_s, "path_flops": path.stats["flops"], "path_bytes": path.stats["bytes"],
                   "max_intermediate": path.stats["max_intermediate_elems"], "n_steps": path.stats["n_steps"],
                   "n_small_steps": path.stats["n_small_steps"], "modeled_ms": path.stats["modeled_seconds"] * 1e3},
        "path_tflops": path.stats["flops"] / (ms * 1e-3) / 1e12,
        "roofline": roof,
        "kernels": kernels,
    }

    if not args.no_cpu_baseline or not args.no_check:
        import oracle
        t0 = time.perf_counter()
        psi_ref = oracle.statevector(circ)
        cpu_s = time.perf_counter() - t0
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = {"value": (1 << n) / cpu_s, "unit": "amplitudes/s",
                                      "cores": oracle.num_threads(), "kind": "oracle",
                                      "sample": "one full statevector of the same circuit (FP64 gate-by-gate, "
                                                f"{len(circ.gates)} gates), {cpu_s:.1f} s"}
        if not args.no_check:
            got = out[0].cpu().numpy().astype(np.complex128)
            result["rel_err_vs_oracle"] = float(np.linalg.norm(got - psi_ref) / np.linalg.norm(psi_ref))
    print(json.dumps(result))


if __name__ == "__main__":
    main()
