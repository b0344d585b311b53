"""GPU parity for QAOA Max-Cut energies and adjoint gradients.

Against the oracle's energy and its own adjoint gradient (complex128, gate by
gate) with |g_gpu - g_oracle| <= 1e-9 and |E_gpu - E_oracle| <= 1e-10; against
the p = 1 ring closed form; and against central finite differences of the GPU
forward within the rounding-limited bound of the difference quotient.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W
from gpu_util import record, require_gpu

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-9
E_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _problem(n, edges, p, w=None):
    from paper_2001_10554_amd.qsim import Qaoa
    return Qaoa(n, edges, p, w)


def _graph(n, seed):
    return W.random_regular_graph(n, 3, seed) if n % 2 == 0 and n >= 4 else W.ring_graph(n)


# (13, 1) and (14, 3): plain passes with RX on wave bits but none on the upper
# lane bits (the backward without the third layout at the end); the other
# sizes cover the plain and merged passes that end lambda in the third layout.
@pytest.mark.parametrize("n,p", [(2, 1), (3, 2), (4, 1), (6, 3), (8, 2), (11, 2), (12, 3), (13, 1), (13, 2), (14, 3), (16, 2), (18, 2),
                                 (19, 1), (20, 2), (22, 1)])
def test_energy_and_gradient_vs_oracle(n, p):
    import torch
    edges = _graph(n, seed=100 + n)
    theta = W.qaoa_angles(p, seed=200 + n)
    prob = _problem(n, edges, p)
    E, G = prob.run(torch.tensor(theta, device="cuda"))
    e_ref, g_ref = oracle.qaoa_grad(n, edges, p, theta)
    record("E", abs(E.item() - e_ref), E_TOL)
    record("gradient", float(np.max(np.abs(G.cpu().numpy()[0] - g_ref))), GRAD_TOL)
    E2, _ = prob.run(torch.tensor(theta, device="cuda"), grad=False)
    record("E", abs(E2.item() - e_ref), E_TOL)


@pytest.mark.parametrize("n", [10, 16, 20])
def test_weighted_graph(n):
    """Real edge weights (per-amplitude phases): one qubit group at 10 qubits,
    two groups with merged layer boundaries at 16 and 20."""
    import torch
    p = 2
    edges = W.random_regular_graph(n, 3, seed=5)
    w = np.linspace(0.25, 2.0, len(edges))
    theta = W.qaoa_angles(p, seed=6)
    E, G = _problem(n, edges, p, w).run(torch.tensor(theta, device="cuda"))
    e_ref, g_ref = oracle.qaoa_grad(n, edges, p, theta, w=w)
    record("E", abs(E.item() - e_ref), E_TOL)
    record("gradient", float(np.max(np.abs(G.cpu().numpy()[0] - g_ref))), GRAD_TOL)


def test_batch_of_angle_sets():
    import torch
    n, p, B = 14, 3, 5
    edges = W.random_regular_graph(n, 3, seed=3)
    thetas = W.qaoa_angles(p, seed=4, hi=2 * math.pi, count=B)
    E, G = _problem(n, edges, p).run(torch.tensor(thetas, device="cuda"))
    for b in range(B):
        e_ref, g_ref = oracle.qaoa_grad(n, edges, p, thetas[b])
        record("E", abs(E[b].item() - e_ref), E_TOL)
        record("gradient", float(np.max(np.abs(G[b].cpu().numpy() - g_ref))), GRAD_TOL)


@pytest.mark.parametrize("n", [6, 12, 15])
def test_p1_ring_closed_form(n):
    import torch
    ring = W.ring_graph(n)
    gamma, beta = 0.41, 1.13
    E, G = _problem(n, ring, 1).run(torch.tensor([gamma, beta], device="cuda", dtype=torch.float64))
    assert abs(E.item() - n * (0.5 + 0.25 * math.sin(4 * beta) * math.sin(2 * gamma))) < 1e-12
    g = G.cpu().numpy()[0]
    assert abs(g[0] - 0.5 * n * math.sin(4 * beta) * math.cos(2 * gamma)) < 1e-11
    assert abs(g[1] - n * math.cos(4 * beta) * math.sin(2 * gamma)) < 1e-11


def test_autograd_function():
    import torch
    from paper_2001_10554_amd.qsim import QAOAEnergy
    n, p = 10, 2
    edges = W.random_regular_graph(n, 3, seed=9)
    prob = _problem(n, edges, p)
    th = torch.tensor(W.qaoa_angles(p, seed=10), device="cuda", requires_grad=True)
    E = QAOAEnergy.apply(th, prob)
    (3.0 * E).backward()
    _, g_ref = oracle.qaoa_grad(n, edges, p, th.detach().cpu().numpy())
    record("autograd gradient / 3", float(np.max(np.abs(th.grad.cpu().numpy() / 3.0 - g_ref))), GRAD_TOL)


def test_config3_24q_p8_vs_oracle_and_fd():
    """QAOA Max-Cut, 24 qubits, random 3-regular graph, p = 8, angles U[0, pi]:
    adjoint gradient vs the oracle's (<= 1e-9) and vs central differences
    (h = 1e-6) of the same GPU forward, within 10 * (eps_E / h + h^2 |E'''|)."""
    import torch
    n, p, h = 24, 8, 1e-6
    edges = W.random_regular_graph(n, 3, seed=3)
    theta = W.qaoa_angles(p, seed=3)
    prob = _problem(n, edges, p)
    E, G = prob.run(torch.tensor(theta, device="cuda"))
    g = G.cpu().numpy()[0]
    e_ref, g_ref = oracle.qaoa_grad(n, edges, p, theta)
    record("E", abs(E.item() - e_ref), E_TOL)
    record("gradient", float(np.max(np.abs(g - g_ref))), GRAD_TOL)
    shifts = np.repeat(theta[None, :], 4 * p, axis=0)
    for k in range(2 * p):
        shifts[2 * k, k] += h
        shifts[2 * k + 1, k] -= h
    Es, _ = prob.run(torch.tensor(shifts, device="cuda"), grad=False)
    Es = Es.cpu().numpy()
    fd = (Es[0::2] - Es[1::2]) / (2 * h)
    # E ~ 36 in magnitude: rounding of each forward ~ 1e-13 relative -> eps_E/h ~ 4e-6 / ... bound:
    tau = 10 * (abs(E.item()) * 1e-14 / h + h * h * 1e3)
    record("|g_adjoint - g_FD| (h = 1e-6)", float(np.max(np.abs(fd - g))), tau)


def test_fd_error_vs_step_has_truncation_and_rounding_branches():
    """Central differences of the GPU forward against the adjoint gradient over
    h = 1e-2 ... 1e-8: the error first falls as h^2 (truncation, so a tenfold
    smaller h gives about a hundredfold smaller error) and then grows as eps/h
    (rounding), with the adjoint inside the valley."""
    import torch
    n, p = 14, 3
    edges = W.random_regular_graph(n, 3, seed=6)
    theta = W.qaoa_angles(p, seed=6)
    prob = _problem(n, edges, p)
    _, G = prob.run(torch.tensor(theta, device="cuda"))
    g = G.cpu().numpy()[0]
    hs = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8]
    err = []
    for h in hs:
        shifts = np.repeat(theta[None, :], 4 * p, axis=0)
        for k in range(2 * p):
            shifts[2 * k, k] += h
            shifts[2 * k + 1, k] -= h
        Es, _ = prob.run(torch.tensor(shifts, device="cuda"), grad=False)
        Es = Es.cpu().numpy()
        err.append(np.abs((Es[0::2] - Es[1::2]) / (2 * h) - g))
    err = np.array(err)  # [h, component]
    big = err[0] > 1e-6  # components whose truncation term is well above rounding at h = 1e-2
    assert big.any()
    ratio = err[0][big] / err[1][big]
    assert np.all((ratio > 50) & (ratio < 200)), ratio
    worst = err.max(axis=1)
    valley = worst[3:5].min()  # h = 1e-5, 1e-6: the oracle's own curve bottoms out near 1e-8 here
    assert valley < 5e-8
    assert worst[-1] > 10 * valley


_MERGE_CHILD = r"""
import json, sys
import numpy as np
import torch
from paper_2001_10554_amd import workloads as W
from paper_2001_10554_amd.qsim import Qaoa
out = []
for n, p in json.loads(sys.argv[1]):
    edges = W.random_regular_graph(n, 3, seed=n + p)
    theta = W.qaoa_angles(p, seed=n)
    E, G = Qaoa(n, edges, p).run(torch.tensor(theta, device="cuda"))
    out.append([E.item(), G.cpu().numpy()[0].tolist()])
print(json.dumps(out))
"""


@pytest.mark.parametrize("mode", ["0", "1", "2"])
def test_merge_policies_match_oracle(mode):
    """Every layer-boundary policy (never merge, merge every boundary, the
    default that skips the first group) with two and three qubit groups
    (10-qubit tiles force three groups at 20 and 22 qubits)."""
    import json
    import os
    import subprocess
    import sys
    cases = [(16, 3), (20, 4), (22, 2)]
    env = dict(os.environ, QSIM_QAOA_MERGE=mode, QSIM_QAOA_TB="10", QSIM_QAOA_R="3")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _MERGE_CHILD, json.dumps(cases)], env=env, cwd=root, capture_output=True, text=True,
                       timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    got = json.loads(r.stdout.strip().splitlines()[-1])
    for (n, p), (e, g) in zip(cases, got):
        edges = W.random_regular_graph(n, 3, seed=n + p)
        theta = W.qaoa_angles(p, seed=n)
        e_ref, g_ref = oracle.qaoa_grad(n, edges, p, theta)
        record(f"E ({mode}, n={n}, p={p})", abs(e - e_ref), E_TOL)
        record(f"gradient ({mode}, n={n}, p={p})", float(np.max(np.abs(np.array(g) - g_ref))), GRAD_TOL)
