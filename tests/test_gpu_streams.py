"""Calls queued on a stream other than torch's current one: the binding orders
the call after the current stream's queued work (its inputs), allocates its
workspace and outputs on the call's stream, and makes the current stream wait
before the outputs are read.  Results must equal the same calls on the
current stream bit for bit (same kernels, same launch shapes)."""
import math

import numpy as np
import pytest

from paper_2001_10554_amd import workloads as W
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_side_stream_results_equal_current_stream():
    import torch
    from paper_2001_10554_amd.qsim import Pool, Qaoa, State, traj_run
    side = torch.cuda.Stream()

    # trajectories
    n, gates = 10, W.qft_circuit(10)
    ref = traj_run(n, gates, 5, 64, 0.01, 3, log_cap=8)
    got = traj_run(n, gates, 5, 64, 0.01, 3, log_cap=8, stream=side)
    for k in ref:
        assert torch.equal(ref[k], got[k]), k

    # QAOA: the angles are produced on the current stream just before the call
    edges = W.random_regular_graph(12, 3, seed=1)
    q = Qaoa(12, edges, 2)
    th = torch.tensor(W.qaoa_angles(2, seed=2, count=3), device="cuda")
    E0, G0 = q.run(th)
    th2 = th * 1.0
    E1, G1 = q.run(th2, stream=side)
    assert torch.equal(E0, E1) and torch.equal(G0, G1)

    # pool
    graphs = [W.random_regular_graph(m, 3, seed=m) for m in (8, 10)]
    pool = Pool(graphs, [8, 10], 2, 2)
    a = torch.tensor(W.qaoa_angles(2, seed=3, hi=2 * math.pi, count=pool.count), device="cuda")
    E0 = pool.run(a)[0].clone()
    E1 = pool.run(a * 1.0, stream=side)[0].clone()
    assert torch.equal(E0, E1)

    # a state on the side stream, read on the current one
    s0 = State(14).init_random(4)
    s1 = State(14, stream=side).init_random(4)
    m = W.haar_list(5, 1)[0]
    s0.apply_1q(13, m)
    s1.apply_1q(13, m)
    assert torch.equal(s0.expect_z_all(), s1.expect_z_all())
    assert torch.equal(s0.sample(1000, 9), s1.sample(1000, 9))
    side.synchronize()
    assert np.array_equal(s0.amps.cpu().numpy(), s1.amps.cpu().numpy())
