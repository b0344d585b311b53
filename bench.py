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
summed kernel time.  roofline = the same for the dominant kernels (the
one-qubit gate: k_apply_1q, and k_apply_1q_lane for targets below 6) against
MI355X's 8 TB/s.  cpu_baseline = the CPU oracle on a bounded sample of the
same sweep.  The line ends with both halves of the metric: the QAOA
adjoint/finite-difference ratio and the per-target minima.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1q-gate HBM GB/s (% roofline) at 32q c128; QAOA adjoint grads/s vs finite-diff"
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32, help="qubits of the sweep register")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the QAOA, pool and trajectory measurements")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_1q_32q_c128.json"))
    ap.add_argument("--section", choices=sorted(SECTIONS), help="run only this extra section and print its JSON")
    ap.add_argument("--curves", default=None,
                    help="also compute the convergence / approximation-ratio curves of the study workloads and write them "
                         "to this JSON file (they are not part of the printed line)")
    return ap.parse_args()


CURVES = {}  # filled by the sections when --curves is given


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
    # Reference: a plain device-to-device copy of the register (known size,
    # also the scale for the HBM byte counters).
    dst = torch.empty_like(s.amps)
    copy_t = []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(s.amps)
        b.record(stream)
        b.synchronize()
        copy_t.append(a.elapsed_time(b) * 1e-3)
    copy_gbs = 2 * (16 << n) / min(copy_t) / 1e9
    del dst
    # The same sweep as one fused block on the same register: read+write
    # passes instead of one pass per gate.
    from paper_2001_10554_amd.qsim import block_passes
    gates = W.gates_array([W.gate(W.G_1Q, q, -1, m) for q, m in enumerate(mats)]
                          + [W.gate(W.G_C1Q, c, t, X) for c, t in cnots])
    log("timing the sweep as one fused block")
    t_fused = _time_cuda(lambda: s.apply_block(gates), 2)
    passes = block_passes(n, gates)
    gate_by_gate = sum(statistics.median(v) for v in per_1q.values()) + sum(statistics.median(v) for v in per_cx.values())
    fused = {"workload": f"the same {n}-qubit sweep ({len(gates)} gates) as one fused block", "passes": passes,
             "ms": round(t_fused * 1e3, 3), "pass_GB_per_s": round(passes * 2 * (16 << n) / t_fused / 1e9, 1),
             "pass_frac": round(passes * 2 * (16 << n) / t_fused / 1e9 / PEAK_HBM_GBS, 4),
             "gate_by_gate_ms": round(gate_by_gate * 1e3, 3), "speedup": round(gate_by_gate / t_fused, 2)}
    del s
    torch.cuda.empty_cache()
    return wall, per_1q, per_cx, norm, copy_gbs, fused


def _time_cuda(fn, reps):
    import torch
    st = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        fn()
    b.record(st)
    b.synchronize()
    return a.elapsed_time(b) * 1e-3 / reps


def qaoa_bench():
    """QAOA Max-Cut, 24 qubits, random 3-regular graph, p = 8, angles U[0, pi]:
    adjoint gradient evaluations/s vs central finite differences (h = 1e-6,
    2 * 2p forward evaluations per gradient, batched through the same fused
    forward) on the same GPU."""
    import numpy as np
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import Qaoa
    n, p, h = 24, 8, 1e-6
    edges = W.random_regular_graph(n, 3, seed=3)
    theta = torch.tensor(W.qaoa_angles(p, seed=3), device="cuda")
    prob = Qaoa(n, edges, p)
    t_adj = _time_cuda(lambda: prob.run(theta, grad=True), 10)
    E, G = prob.run(theta, grad=True)
    shifts = theta.repeat(4 * p, 1)
    idx = torch.arange(2 * p, device="cuda")
    shifts[2 * idx, idx] += h
    shifts[2 * idx + 1, idx] -= h
    # FD forwards in one batched call (workspace for all 4p angle sets at once).
    prob._ws[False] = torch.empty(prob.workspace(False).numel() * 4 * p, dtype=torch.uint8, device="cuda")
    t_fd = _time_cuda(lambda: prob.run(shifts, grad=False), 3)
    Es, _ = prob.run(shifts, grad=False)
    fd = (Es[0::2] - Es[1::2]) / (2 * h)
    g = G[0]
    out = {"workload": "QAOA Max-Cut, 24 qubits, random 3-regular graph (seed 3), p=8, angles U[0,pi] (seed 3), complex128",
           "adjoint_grads_per_s": round(1.0 / t_adj, 2), "adjoint_ms": round(t_adj * 1e3, 3),
           "fd_grads_per_s": round(1.0 / t_fd, 2), "fd_ms": round(t_fd * 1e3, 3),
           "ratio": round(t_fd / t_adj, 2), "E": E.item(), "max_abs_adj_minus_fd": float(torch.max(torch.abs(g - fd)).item())}
    del prob
    torch.cuda.empty_cache()
    return out


def pool_bench(reps=2):
    """Pool: 256 QAOA Max-Cut graphs (qubit counts uniform over {14,...,22},
    random 3-regular), p = 4, 64 swarm-style angle sets per graph in [0, 2pi):
    all 16,384 <C> values and adjoint gradients per replay of the captured graph."""
    import numpy as np
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import Pool
    w = W.pool_workload(256, 64, 4, seed=4)
    # The autotuner appends its choice per size class ("n:p:sets:grad TB r") to this file.
    fd, tune_path = tempfile.mkstemp(suffix=".txt")
    os.close(fd)
    os.unlink(tune_path)
    os.environ["QSIM_AUTOTUNE_CACHE"] = tune_path
    pool = Pool(w.graphs, w.n_qubits, 64, 4)
    a = torch.tensor(np.concatenate(w.angles), device="cuda")
    t0 = time.perf_counter()
    pool.run(a)  # plans, autotunes, captures
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    t = _time_cuda(lambda: pool.run(), reps)
    tuned = {}
    if os.path.exists(tune_path):
        for line in open(tune_path):
            key, tb, r = line.split()
            tuned[int(key.split(":")[0])] = (int(tb), int(r))
        os.unlink(tune_path)
    del os.environ["QSIM_AUTOTUNE_CACHE"]
    # State transfers per circuit over its np passes: forward 2 per pass (the
    # first only writes), backward 3 per pass (checkpoint, lambda in, lambda
    # out; the last pass computes lambda, the first stores none): 5 np - 3.
    # With P qubit groups, layer boundaries are merged passes: np = p(P-1) + 1.
    p = 4
    moved = 0
    for n in w.n_qubits:
        tb, r = tuned.get(n, (min(n, 12), 3))
        P = 1 if n <= tb else 1 + -(-(n - tb) // (tb - r))
        npass = p * (P - 1) + 1 if P >= 2 else p
        moved += 64 * (5 * npass - 3) * (1 << n) * 16  # 64 angle sets per graph
    out = {"workload": "pool: 256 graphs x 64 angle sets, n ~ U{14..22}, p=4, complex128, E + gradients",
           "circuits": pool.count, "seconds_per_pool": round(t, 4), "circuits_per_s": round(pool.count / t, 1),
           "gradients_per_s": round(pool.count / t, 1), "setup_s": round(t_setup, 2),
           "workspace_GiB": round(pool.ws.numel() / 2**30, 2),
           "autotuned_TB_r_by_n": {str(k): list(v) for k, v in sorted(tuned.items())},
           "state_GB_moved": round(moved / 1e9, 1), "effective_GB_per_s": round(moved / t / 1e9, 1),
           "finite": bool(torch.isfinite(pool.E).all().item())}
    del pool
    torch.cuda.empty_cache()
    return out


def traj_bench():
    """Noise ensemble: 16-qubit QFT on a seeded basis state, depolarizing p = 1e-3
    per touched qubit as stochastic Pauli insertions, 1024 trajectories."""
    import numpy as np
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import traj_run
    n, T, p = 16, 1024, 1e-3
    gates = W.qft_circuit(n)
    x0 = W.random_basis_index(n, 5)
    out = {"workload": "16-qubit QFT on a seeded basis state, depolarizing p=1e-3, 1024 trajectories"}
    Ts = [1 << k for k in range(11)]
    for name, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        t = _time_cuda(lambda: traj_run(n, gates, x0, T, p, seed=5, dtype=dt, prob_mean=True), 3)
        r = traj_run(n, gates, x0, T, p, seed=5, dtype=dt)
        fid = r["fid"].cpu().numpy()
        out[name] = {"trajectories_per_s": round(T / t, 1), "ms": round(t * 1e3, 3), "mean_fidelity": float(fid.mean()),
                     "max_abs_Z": float(r["z"].abs().max().item()),
                     "max_abs_p_minus_2^-16": float((r["prob_mean"] - 2.0 ** -n).abs().max().item()),
                     "insertions": int(r["counts"].sum().item())}
    if CURVES.get("enabled"):
        # Convergence of the trajectory means with T, over 8 independent seeds (c128).
        curves_f, curves_x = [], []
        for seed in range(5, 13):
            r = traj_run(n, gates, x0, T, p, seed=seed, dtype=torch.complex128, prob_mean=False)
            fid = r["fid"].cpu().numpy()
            xm = r["x"].cpu().numpy().mean(axis=1)  # mean over qubits of <X_q>, per trajectory
            curves_f.append([round(float(fid[:k].mean()), 6) for k in Ts])
            curves_x.append([round(float(xm[:k].mean()), 6) for k in Ts])
        CURVES["traj_convergence"] = {"T": Ts, "seeds": list(range(5, 13)), "mean_fidelity": curves_f, "mean_X": curves_x}
    return out


def brick_bench():
    """12-qubit complex128 brick circuit from |0>: 20 layers of Haar 1q gates on
    every qubit and CZ on brick pairs (350 gates) as one fused block, then all
    <Z_i>.  The register fits one 64 KiB tile, so the block is one launch."""
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import State
    n = 12
    gates = W.brick_circuit(n, 20, seed=1)
    s = State(n, torch.complex128)

    def run():
        s.init_basis(0)
        s.apply_block(gates)
        s.expect_z_all()
    t = _time_cuda(run, 20)
    return {"workload": "12-qubit complex128 brick circuit, 20 layers, 350 gates, fused block + <Z_i>",
            "us_per_circuit": round(t * 1e6, 1), "gates_per_s": round(len(gates) / t, 1)}


def fused_bench(n=30):
    """The sweep's gate list (Haar 1q on q = 0..n-1, then CNOT(q, q+1)) on a
    30-qubit complex128 register (16 GiB) as one fused block, against the same
    gates launched one by one.  pass_GB_per_s: the passes' real read+write
    traffic; gate_GB_per_s: what the gates would move one at a time (1q: the
    whole register, CNOT: the control-1 half, or all of it when the control
    lies inside a 128-byte line), which fusion lets exceed the HBM peak."""
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import State, block_passes
    mats, cnots = W.sweep_circuit(n, seed=2)
    gates = W.gates_array([W.gate(W.G_1Q, q, -1, m) for q, m in enumerate(mats)]
                          + [W.gate(W.G_C1Q, c, t, W.PAULI_X) for c, t in cnots])
    passes = block_passes(n, gates)
    s = State(n, torch.complex128).init_random(2)
    t_fused = _time_cuda(lambda: s.apply_block(gates), 3)

    def one_by_one():
        for q, m in enumerate(mats):
            s.apply_1q(q, m)
        for c, t in cnots:
            s.apply_c1q(c, t, W.PAULI_X)
    t_single = _time_cuda(one_by_one, 2)
    amp = 16
    full = 2 * (1 << n) * amp
    gate_bytes = n * full + sum(full if c < 3 else full // 2 for c, _ in cnots)
    del s
    torch.cuda.empty_cache()
    return {"workload": f"{n}-qubit complex128 sweep (Haar 1q on every qubit, CNOT chain) as one fused block",
            "gates": int(len(gates)), "passes": passes, "ms": round(t_fused * 1e3, 3),
            "pass_GB_per_s": round(passes * full / t_fused / 1e9, 1),
            "gate_GB_per_s": round(gate_bytes / t_fused / 1e9, 1),
            "one_by_one_ms": round(t_single * 1e3, 3), "speedup": round(t_single / t_fused, 2)}


def pso_bench(G=300, R=16, rounds=32):
    """Particle swarm over the pool, the paper's study shape: random 3-regular
    graphs on 18 vertices, p = 4 (8 coordinates), one swarm of R particles per
    graph, R * rounds = 512 evaluations per graph, eq. (4) with the paper's
    constants.  The whole run (pool evaluations + swarm kernels) stays on the
    device; the approximation ratio divides by the exact Max-Cut value."""
    import numpy as np
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import Pool, Swarm, cut_max
    n, p = 18, 4
    graphs = [W.random_regular_graph(n, 3, seed=1000 + g) for g in range(G)]
    sizes = [n] * G
    t0 = time.perf_counter()
    mx, _ = cut_max(graphs, sizes)
    torch.cuda.synchronize()
    t_cut = time.perf_counter() - t0
    pool = Pool(graphs, sizes, R, p, grad=False, ws_circuits=G * R)
    sw = Swarm(pool)
    t0 = time.perf_counter()
    sw.run(rounds, seed=1)  # plans, tunes and captures the pool on first use
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    t = _time_cuda(lambda: sw.run(rounds, seed=2), 2)
    hist = sw.run(rounds, seed=3)
    ratio = (hist / mx[None, :]).cpu().numpy()
    evals = G * R * rounds
    out = {"workload": f"particle swarm: {G} random 3-regular graphs, n={n}, p={p}, {R} particles x {rounds} rounds "
                       f"(512 evaluations per graph), complex128",
           "evaluations_per_s": round(evals / t, 1), "ms_per_round": round(t / rounds * 1e3, 3), "seconds_per_run": round(t, 4),
           "first_run_s": round(t_setup, 2), "cut_max_ms_all_graphs": round(t_cut * 1e3, 2),
           "mean_ratio_at_512_evals": round(float(ratio[-1].mean()), 5), "std_ratio_at_512_evals": round(float(ratio[-1].std()), 5),
           "max_ratio": round(float(ratio.max()), 5)}
    if CURVES.get("enabled"):
        CURVES["pso_mean_ratio_by_round"] = [round(float(x), 5) for x in ratio.mean(axis=1)]
    del pool, sw
    torch.cuda.empty_cache()
    return out


def noise_bench(T=1024):
    """Noisy QAOA (the paper's convergence study shape): 16-qubit random
    3-regular graph, p = 4; angles from a particle swarm on the device
    (32 particles, 48 rounds) and, for the second panel, uniform random angles;
    a noise gate of one gate time on every touched qubit after every gate,
    T1 = 500, T2 = 250 gate times; <C> per trajectory as a diagonal read-out.
    Convergence of the ensemble mean of <C> with the ensemble size for 8
    random streams."""
    import numpy as np
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import Pool, Swarm, cut_max, traj_run
    n, p = 16, 4
    edges = W.random_regular_graph(n, 3, seed=8)
    e_exact = cut_max([edges], [n])[0].item()
    pool = Pool([edges], [n], 32, p, grad=False, ws_circuits=32)
    sw = Swarm(pool)
    hist = sw.run(48, seed=8)
    theta_pso = sw.gbest[0].cpu().numpy()
    e_pso = float(hist[-1, 0].item())
    k = np.arange(1 << n)
    diag = torch.tensor(sum(((k >> u) ^ (k >> v)) & 1 for u, v in edges).astype(np.float64), device="cuda")
    Ts = [1 << j for j in range(int(math.log2(T)) + 1)]
    out = {"workload": f"noisy QAOA: 16 qubits, random 3-regular graph (seed 8), p={p}, noise gate of 1 gate time per touched "
                       f"qubit after every gate, T1=500, T2=250, {T} trajectories, complex128",
           "E_exact": e_exact}
    for label, theta in (("pso_angles", theta_pso), ("random_angles", W.qaoa_angles(p, seed=9, hi=2 * math.pi))):
        gates = W.with_noise_gates(W.qaoa_circuit(n, edges, p, theta), 1.0)
        # per-trajectory <C> (the diagonal read-out) only: no <Z_q>, <X_q>, fidelity
        run = lambda seed: traj_run(n, gates, 0, T, 0.0, seed, T1=500.0, T2=250.0, diag=diag, prob_mean=False,  # noqa: E731
                                    readouts=())
        t = _time_cuda(lambda: run(1), 2)
        r = run(1)
        ideal = traj_run(n, gates, 0, 1, 0.0, 1, diag=diag, prob_mean=False)  # no decay: the noiseless value
        out[label] = {"gates": int(len(gates)), "trajectories_per_s": round(T / t, 1), "ms": round(t * 1e3, 3),
                      "noiseless_C": round(float(ideal["diag"][0].item()), 6),
                      "noisy_C_mean": round(float(r["diag"].mean().item()), 5)}
        if CURVES.get("enabled"):
            curves = []
            for seed in range(1, 9):
                c = run(seed)["diag"].cpu().numpy()
                curves.append([round(float(c[:m].mean()), 5) for m in Ts])
            CURVES[f"noise_{label}_convergence"] = {"T": Ts, "mean_C": curves}
    out["pso_angles"]["swarm_best_C"] = round(e_pso, 6)
    del pool, sw
    torch.cuda.empty_cache()
    return out


def readout_bench(n=30):
    """Every single-state row at 30 qubits complex128 (16 GiB), as effective
    HBM GB/s of the algorithmic bytes: initialisation, the cost layer, the
    two-qubit diagonal and SWAP gates, the read-outs and sampling."""
    import numpy as np
    import torch

    from paper_2001_10554_amd import workloads as W
    from paper_2001_10554_amd.qsim import State
    S = (1 << n) * 16
    s = State(n).init_random(1)
    t2 = State(n).init_random(2)
    edges = W.random_regular_graph(n, 3, seed=3)
    diag = torch.rand(1 << n, dtype=torch.float64, device="cuda")
    cz = np.array([1, 1, 1, -1], dtype=np.complex128)
    out = {"workload": f"{n}-qubit complex128 register (16 GiB), seeded random state; random 3-regular graph for the cut"}

    def rate(name, fn, nbytes, reps=3, **extra):
        t = _time_cuda(fn, reps)
        out[name] = {"ms": round(t * 1e3, 3), "GB_per_s": round(nbytes / t / 1e9, 1), **extra}

    rate("init_basis", lambda: s.init_basis(5), S)                      # write every amplitude
    rate("init_uniform", lambda: s.init_uniform(), S)
    rate("init_random", lambda: s.init_random(1), 4 * S)                # write, read for the norm, read + write to scale
    rate("cut_phase", lambda: s.apply_cut_phase(edges, 0.3), 2 * S)
    rate("diag2_cz", lambda: s.apply_diag2(3, 17, cz), 2 * S // 4)      # only the |11> quarter moves
    rate("swap", lambda: s.apply_swap(5, 25), 2 * S // 2)               # the (1,0)/(0,1) quarters, whole lines
    rate("swap_in_line", lambda: s.apply_swap(2, 25), 2 * S)            # qubit 2 inside the 128-byte line: every line moves
    rate("expect_z_all", lambda: s.expect_z_all(), S)
    rate("norm2", lambda: s.norm2(), S)
    rate("prob_one", lambda: s.prob_one(7), S)
    rate("expect_cut", lambda: s.expect_cut(edges), S)
    rate("expect_diag", lambda: s.expect_diag(diag), S + (1 << n) * 8)
    rate("expect_pauli_xyz", lambda: s.expect_pauli(0b1010101, 0b1100011), S)
    rate("inner", lambda: s.inner(t2), 2 * S)
    shots = 1 << 20
    t = _time_cuda(lambda: s.sample(shots, 11), 3)
    out["sample"] = {"shots": shots, "ms": round(t * 1e3, 3), "shots_per_s": round(shots / t, 1),
                     "GB_per_s_of_state": round(S / t / 1e9, 1)}
    del s, t2, diag
    torch.cuda.empty_cache()
    return out


def kq_bench(n=30):
    """Dense k-qubit gates (k = 1..5, random unitaries) and one Born
    measurement on a 30-qubit complex128 register (16 GiB)."""
    import numpy as np
    import torch

    from paper_2001_10554_amd.qsim import State
    s = State(n).init_random(1)
    state_bytes = (1 << n) * 16
    out = {"workload": f"{n}-qubit complex128 register: dense k-qubit gate on qubits [n-1, 0, n/2, 5, 17][:k], one measurement"}
    g = np.random.default_rng(0)
    for k in range(1, 6):
        a = g.standard_normal((1 << k, 1 << k)) + 1j * g.standard_normal((1 << k, 1 << k))
        U, _ = np.linalg.qr(a)
        qs = [n - 1, 0, n // 2, 5, 17][:k]
        t = _time_cuda(lambda: s.apply_kq(qs, U), 3)
        out[f"k{k}"] = {"ms": round(t * 1e3, 3), "GB_per_s": round(2 * state_bytes / t / 1e9, 1),
                        "GFLOP_per_s": round((1 << n) * (1 << k) * 8 / t / 1e9, 1)}
    t = _time_cuda(lambda: s.measure(n // 2, 7), 3)
    # read the state for the two sums, then read the kept half and write all
    out["measure"] = {"ms": round(t * 1e3, 3), "GB_per_s": round(2.5 * state_bytes / t / 1e9, 1)}
    del s
    torch.cuda.empty_cache()
    return out


def cpu_baseline(seconds):
    """The oracle (plain C; OpenMP on its element loops) on bounded samples of
    the workloads: one-qubit gates per target on a 28-qubit register (4 GiB;
    the 32-qubit register does not fit the host budget of this run), with all
    host threads and single-threaded; the QAOA adjoint gradient at 22 qubits,
    p = 8 (one evaluation); the brick circuit, pool circuits and trajectories
    on small samples.  `seconds` caps the single-threaded gate timing."""
    import numpy as np

    import oracle
    from paper_2001_10554_amd import workloads as W

    nthreads = oracle.threads()
    n = 28
    mats, _ = W.sweep_circuit(n, seed=2)
    psi = oracle.init_random(n, 2)
    gate_bytes = 2 * (1 << n) * 16
    per_q = {}
    for q in range(n):
        t = time.perf_counter()
        oracle.apply_1q(psi, q, mats[q])
        per_q[q] = time.perf_counter() - t
    omp_gbs = n * gate_bytes / sum(per_q.values()) / 1e9
    oracle.set_threads(1)
    single, spent = {}, 0.0
    try:
        for q in (0, 7, 14, 21, n - 1):
            if spent > seconds:
                break
            t = time.perf_counter()
            oracle.apply_1q(psi, q, mats[q])
            single[q] = time.perf_counter() - t
            spent += single[q]
    finally:
        oracle.set_threads(nthreads)
    out = {"value": round(omp_gbs, 3), "unit": "GB/s", "cores": nthreads, "kind": "oracle",
           "sample": f"one Haar one-qubit gate on each target q = 0..{n-1} of a {n}-qubit c128 register, "
                     f"{nthreads} OpenMP threads",
           "per_qubit_gbs": {str(q): round(gate_bytes / t / 1e9, 2) for q, t in per_q.items()},
           "single_thread": {"GB_per_s": round(len(single) * gate_bytes / sum(single.values()) / 1e9, 3),
                             "targets": sorted(single)}}
    del psi
    nq, p = 22, 8
    edges = W.random_regular_graph(nq, 3, seed=3)
    theta = W.qaoa_angles(p, seed=3)
    t0 = time.perf_counter()
    oracle.qaoa_grad(nq, edges, p, theta)
    t_adj = time.perf_counter() - t0
    out["qaoa"] = {"adjoint_grads_per_s": round(1.0 / t_adj, 4),
                   "sample": f"oracle adjoint gradient, {nq}-qubit random 3-regular graph, p={p}, one evaluation, "
                             f"{nthreads} threads (24 qubits takes ~4x longer)"}
    gates = W.brick_circuit(12, 20, seed=1)
    t0 = time.perf_counter()
    for _ in range(20):
        psi = oracle.init_basis(12, 0)
        oracle.apply_gates(psi, gates)
        oracle.expect_z_all(psi)
    out["brick12"] = {"us_per_circuit": round((time.perf_counter() - t0) / 20 * 1e6, 1), "sample": "20 circuits"}
    w = W.pool_workload(8, 1, 4, seed=4, n_choices=(14, 16, 18))
    t0 = time.perf_counter()
    for g in range(8):
        oracle.qaoa_grad(w.n_qubits[g], w.graphs[g], 4, w.angles[g][0])
    out["pool"] = {"circuits_per_s": round(8 / (time.perf_counter() - t0), 2),
                   "sample": "8 pool circuits (E + adjoint gradient), n in {14,16,18}, p=4"}
    qft = W.qft_circuit(16)
    x0 = W.random_basis_index(16, 5)
    t0 = time.perf_counter()
    oracle.traj_ensemble(16, qft, x0, 16, 1e-3, seed=5)
    out["traj"] = {"trajectories_per_s": round(16 / (time.perf_counter() - t0), 2),
                   "sample": "16 trajectories of the 16-qubit QFT with read-outs (c128)"}
    return out


SECTIONS = {}  # name -> function, filled below the section definitions


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.section:
        print(json.dumps({"section": args.section, **SECTIONS[args.section]()}), flush=True)
        return
    n = args.n
    wall, per_1q, per_cx, norm, copy_gbs, fused = sweep_bench(n, args.steps, args.warmup)
    bytes_1q = 2 * (1 << n) * 16
    t1q = sum(sum(v) for v in per_1q.values())
    launches_1q = sum(len(v) for v in per_1q.values())
    avg_1q = t1q / launches_1q
    gbs = bytes_1q * launches_1q / t1q / 1e9
    # Per target: the median launch time of the timed steps.
    per_q = {q: round(bytes_1q / statistics.median(v) / 1e9, 1) for q, v in per_1q.items()}
    # CNOT: the control-1 half is read and written (2^(n-1) amplitudes, R+W);
    # a control inside a 128-byte line (c < 3 for c128) touches every line, so
    # its algorithmic bytes are the whole register (line granularity).
    per_c = {}
    for q, v in per_cx.items():
        bytes_cx = 2 * (1 << n) * 16 if q < 3 else 2 * (1 << (n - 1)) * 16
        per_c[q] = round(bytes_cx / statistics.median(v) / 1e9, 1)
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
        "per_qubit_1q_gbs": per_q,
        "per_qubit_cnot_gbs": per_c,
        "device_copy_gbs": round(copy_gbs, 1),
        "value_over_device_copy": round(gbs / copy_gbs, 3),
        "norm_after": norm,
        f"fused{n}": fused,
    }
    if args.curves:
        CURVES["enabled"] = True
    if not args.no_extra:
        for name in ("qaoa", "pool", "traj", "brick12", "fused30", "pso", "rows30", "kq", "noise"):
            log(name)
            out[name] = SECTIONS[name]()
    out["roofline"] = {"bound": "hbm", "achieved": round(bytes_1q / avg_1q / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": round(bytes_1q / avg_1q / 1e9 / PEAK_HBM_GBS, 4), "traffic": traffic,
                       "kernel": "k_apply_1q (targets 6..n-1) + k_apply_1q_lane (targets 0..5)",
                       "bytes_per_launch": bytes_1q, "avg_launch_ms": round(avg_1q * 1e3, 4)}
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    if "qaoa" in out:
        q = out["qaoa"]
        out["qaoa_adjoint_grads_per_s"] = q["adjoint_grads_per_s"]
        out["qaoa_fd_grads_per_s"] = q["fd_grads_per_s"]
        out["qaoa_adjoint_over_fd"] = q["ratio"]
    out["min_1q_frac"] = round(min(per_q.values()) / PEAK_HBM_GBS, 4)
    out["min_cnot_frac"] = round(min(per_c.values()) / PEAK_HBM_GBS, 4)
    if args.curves:
        CURVES.pop("enabled")
        with open(args.curves, "w") as f:
            json.dump(CURVES, f)
    print(json.dumps(out), flush=True)


SECTIONS.update({"qaoa": qaoa_bench, "pool": pool_bench, "traj": traj_bench, "brick12": brick_bench, "fused30": fused_bench,
                 "pso": pso_bench, "rows30": readout_bench, "kq": kq_bench, "noise": noise_bench})

if __name__ == "__main__":
    main()
