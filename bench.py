"""Benchmark: one-qubit-gate HBM bandwidth on a 32-qubit complex128 register.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one sweep of the workload the paper's strong-scaling experiment
times (a random 2x2 gate applied to every qubit of a 32-qubit state): Haar
one-qubit gates on qubits 0..31 in order, then CNOT(q, q+1) for q = 0..30, on
a seeded random normalised state resident in HBM (64 GiB).  Every gate runs as
its own kernel on the state's stream; HIP events around each gate give the
per-launch durations.

Printed: one JSON line.  value = algorithmic bytes of the one-qubit gates
(2 * 2^32 * 16 B each: every amplitude read and written once) divided by their
summed kernel time.  roofline = the same for the dominant kernel (the
one-qubit gate) against MI355X's 8 TB/s.  cpu_baseline = the CPU oracle on a
bounded sample of the same sweep.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1q-gate HBM GB/s (% roofline) at 32q c128; QAOA adjoint grads/s vs finite-diff"
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32, help="qubits of the sweep register")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_1q_32q_c128.json"))
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_bench(n, steps, warmup):
    import numpy as np
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import State

    mats, cnots = W.sweep_circuit(n, seed=2)
    X = W.PAULI_X
    log(f"allocating {n}-qubit c128 register ({(16 << n) / 2**30:.0f} GiB)")
    s = State(n, torch.complex128)
    s.init_random(2)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def one_step(record):
        ev = []
        for q in range(n):
            if record:
                a = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            s.apply_1q(q, mats[q])
            if record:
                b = torch.cuda.Event(enable_timing=True)
                b.record(stream)
                ev.append(("1q", q, a, b))
        for c, t in cnots:
            if record:
                a = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            s.apply_c1q(c, t, X)
            if record:
                b = torch.cuda.Event(enable_timing=True)
                b.record(stream)
                ev.append(("cx", c, a, b))
        return ev

    for _ in range(warmup):
        one_step(False)
    torch.cuda.synchronize()
    log(f"warmup done; timing {steps} steps")
    events = []
    t0 = time.perf_counter()
    for _ in range(steps):
        events += one_step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_1q = {q: [] for q in range(n)}
    per_cx = {q: [] for q in range(n - 1)}
    for kind, q, a, b in events:
        (per_1q if kind == "1q" else per_cx)[q].append(a.elapsed_time(b) * 1e-3)
    norm = s.norm2().item()
    del s
    torch.cuda.empty_cache()
    return wall, per_1q, per_cx, norm


def cpu_baseline(seconds):
    """Oracle (plain C, OpenMP element loops) applying the sweep's Haar gates to a
    smaller register until `seconds` of gate time have been spent."""
    import numpy as np

    import oracle
    from paper_2001_10554_amd import workloads as W

    n = 26
    mats, _ = W.sweep_circuit(n, seed=2)
    psi = oracle.init_random(n, 2)
    spent, gates = 0.0, 0
    q = 0
    while spent < seconds:
        t = time.perf_counter()
        oracle.apply_1q(psi, q, mats[q])
        spent += time.perf_counter() - t
        gates += 1
        q = (q + 1) % n
    bytes_moved = gates * 2 * (1 << n) * 16
    return {"value": round(bytes_moved / spent / 1e9, 3), "unit": "GB/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{gates} one-qubit gates (targets cycling 0..{n-1}) on a {n}-qubit c128 register, "
                      f"{spent:.1f} s of gate time"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n = args.n
    wall, per_1q, per_cx, norm = sweep_bench(n, args.steps, args.warmup)
    bytes_1q = 2 * (1 << n) * 16
    t1q = sum(sum(v) for v in per_1q.values())
    launches_1q = sum(len(v) for v in per_1q.values())
    avg_1q = t1q / launches_1q
    gbs = bytes_1q * launches_1q / t1q / 1e9
    per_q = {q: round(bytes_1q / (sum(v) / len(v)) / 1e9, 1) for q, v in per_1q.items()}
    # CNOT: only the control-1 half is read and written (2^(n-1) amplitudes, R+W).
    bytes_cx = 2 * (1 << (n - 1)) * 16
    per_c = {q: round(bytes_cx / (sum(v) / len(v)) / 1e9, 1) for q, v in per_cx.items()}
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            t = json.load(open(args.traffic_json))
            if t.get("n") == n:
                traffic = t.get("bytes_per_launch")
        except Exception:
            traffic = None
    out = {
        "metric": METRIC,
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{n}-qubit complex128 sweep: Haar 1q gate on q=0..{n-1}, then CNOT(q,q+1) for q=0..{n-2}; "
                               "seeded random normalised state in HBM",
                   "n_qubits": n, "state_bytes": (1 << n) * 16, "gates_per_step": 2 * n - 1},
        "roofline": {"bound": "hbm", "achieved": round(bytes_1q / avg_1q / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(bytes_1q / avg_1q / 1e9 / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": "k_apply_1q", "bytes_per_launch": bytes_1q, "avg_launch_ms": round(avg_1q * 1e3, 4)},
        "per_qubit_1q_gbs": per_q,
        "per_qubit_cnot_gbs": per_c,
        "min_1q_frac": round(min(per_q.values()) / PEAK_HBM_GBS, 4),
        "norm_after": norm,
    }
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
