"""Pins for the oracle's Max-Cut optimum and particle-swarm steps.

The exact cut is checked against graphs whose maximum cut is known in closed
form and against a numpy enumeration written here; the swarm against
geometric invariants of eq. (4) (each attraction term moves a particle along
the line to its best, with the sign the form prescribes), its bookkeeping
invariants, convergence on a concave quadratic with a known maximiser, and
the p = 1 ring, whose best QAOA energy is 3n/4 in closed form.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W

PETERSEN = [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4), (0, 5), (1, 6), (2, 7), (3, 8), (4, 9),
            (5, 7), (7, 9), (6, 9), (6, 8), (5, 8)]


def brute_cut_max(n, edges, w=None):
    k = np.arange(1 << n, dtype=np.int64)
    e = np.asarray(edges).reshape(-1, 2)
    w = np.ones(len(e)) if w is None else np.asarray(w, dtype=np.float64)
    c = np.zeros(1 << n)
    for (u, v), we in zip(e, w):
        c += we * (((k >> u) ^ (k >> v)) & 1)
    return c.max(), int(np.argmax(c))


def test_cut_max_closed_forms():
    complete = lambda n: [(i, j) for i in range(n) for j in range(i + 1, n)]
    assert oracle.cut_max(4, complete(4))[0] == 4
    for n in range(3, 9):
        assert oracle.cut_max(n, complete(n))[0] == (n * n) // 4
    for n in range(3, 13):
        assert oracle.cut_max(n, W.ring_graph(n))[0] == (n if n % 2 == 0 else n - 1)
    k33 = [(a, b) for a in range(3) for b in range(3, 6)]
    assert oracle.cut_max(6, k33)[0] == 9
    assert oracle.cut_max(10, PETERSEN)[0] == 12
    # positive weights on a bipartite graph: every edge is cut
    w = np.linspace(0.5, 2.0, 9)
    assert abs(oracle.cut_max(6, k33, w)[0] - w.sum()) < 1e-12


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cut_max_vs_enumeration(seed):
    g = np.random.default_rng(seed)
    n = 12
    edges = W.random_regular_graph(n, 3, seed)
    best, arg = oracle.cut_max(n, edges)
    bb, ba = brute_cut_max(n, edges)
    assert best == bb and arg == ba
    assert arg < (1 << (n - 1))  # complement symmetry: the smallest maximiser has the top bit clear
    assert oracle.cut_value(arg, edges) == best
    w = g.uniform(0.1, 1.0, len(edges))
    best, arg = oracle.cut_max(n, edges, w)
    bb, ba = brute_cut_max(n, edges, w)
    assert abs(best - bb) < 1e-12 and arg == ba


def test_pso_init_uniform_and_seeded():
    a = oracle.pso_init(4, 16, 8, seed=7)
    b = oracle.pso_init(4, 16, 8, seed=7)
    c = oracle.pso_init(4, 16, 8, seed=8)
    for key in ("pos", "vel"):
        x = a[key]
        assert np.array_equal(x, b[key]) and not np.array_equal(x, c[key])
        assert x.min() >= 0.0 and x.max() < 2 * math.pi
        assert abs(x.mean() - math.pi) < 0.2  # 512 draws: sd of the mean ~ 0.08
        assert len(np.unique(x)) == x.size
    assert not np.array_equal(a["pos"], a["vel"])
    assert np.all(a["pbest_val"] == -np.inf) and np.all(a["gbest_val"] == -np.inf)


def _swarm_with_bests(seed=3, G=2, R=5, D=4):
    sw = oracle.pso_init(G, R, D, seed)
    g = np.random.default_rng(seed)
    sw["pbest"] = g.uniform(0, 6, (G, R, D))
    sw["pbest_val"] = g.uniform(0, 1, (G, R))
    sw["gbest"] = g.uniform(0, 6, (G, D))
    sw["gbest_val"] = np.full(G, 2.0)
    return sw


@pytest.mark.parametrize("attract", [1, -1])
def test_pso_each_term_moves_along_its_line(attract):
    """With only one attraction term active, the step is a multiple in
    [0, phi] of (best - theta) for the standard form, of (theta - best) for
    the printed one; with none active, the velocity decays by omega."""
    for which in ("p", "g", "none"):
        sw = _swarm_with_bests()
        th0, v0 = sw["pos"].copy(), sw["vel"].copy()
        prm = dict(omega=0.0 if which != "none" else 0.66, phi_p=1.6 if which == "p" else 0.0,
                   phi_g=0.62 if which == "g" else 0.0)
        oracle.pso_move(sw, 0, seed=3, attract=attract, **prm)
        step = sw["pos"] - th0
        assert np.allclose(step, sw["vel"], rtol=0, atol=1e-15)
        if which == "none":
            assert np.allclose(sw["vel"], 0.66 * v0, rtol=1e-15, atol=0)
            continue
        target = sw["pbest"] if which == "p" else np.broadcast_to(sw["gbest"][:, None, :], th0.shape)
        d = target - th0
        phi = prm["phi_p"] if which == "p" else prm["phi_g"]
        for gi in range(d.shape[0]):
            for k in range(d.shape[1]):
                coef = np.dot(step[gi, k], d[gi, k]) / np.dot(d[gi, k], d[gi, k])
                assert np.allclose(step[gi, k], coef * d[gi, k], rtol=0, atol=1e-12)  # collinear
                assert 0.0 < attract * coef <= phi
    # different particles and rounds draw different r values
    sw = _swarm_with_bests()
    th0 = sw["pos"].copy()
    oracle.pso_move(sw, 0, seed=3, omega=0.0, phi_p=1.6, phi_g=0.0)
    coefs = [(sw["pos"][0, k] - th0[0, k])[0] / (sw["pbest"][0, k] - th0[0, k])[0] for k in range(5)]
    assert len(set(np.round(coefs, 12))) == 5


def test_pso_bests_are_running_maxima():
    g = np.random.default_rng(5)
    sw = oracle.pso_init(3, 6, 2, seed=5)
    seen = np.full((3, 6), -np.inf)
    hist = []
    for r in range(8):
        E = g.normal(size=(3, 6))
        E[1, 2] = E[1, 4] = 9.0 if r == 3 else E[1, 2]  # a tie: the lower index wins
        oracle.pso_update_bests(sw, E)
        seen = np.maximum(seen, E)
        assert np.array_equal(sw["pbest_val"], seen)
        assert np.array_equal(sw["gbest_val"], seen.max(axis=1))
        hist.append(sw["gbest_val"].copy())
        if r == 3:
            assert np.array_equal(sw["gbest"][1], sw["pbest"][1, 2])
        oracle.pso_move(sw, r, seed=5)
    assert np.all(np.diff(np.array(hist), axis=0) >= 0)


def test_pso_converges_on_concave_quadratic():
    """max of -|theta - c|^2 is at c; the standard form with the paper's
    constants finds it, the printed sign does not."""
    c = np.array([1.0, 2.5, 4.0, 0.5])
    f = lambda pos: -np.sum((pos - c) ** 2, axis=-1)
    sw, hist, _ = oracle.pso_run(f, 2, 16, 4, rounds=150, seed=11)
    assert np.all(hist[-1] > -1e-8)
    assert np.allclose(sw["gbest"], c, atol=1e-4)
    sw_m, hist_m, _ = oracle.pso_run(f, 2, 16, 4, rounds=30, seed=11, attract=-1)
    assert np.all(hist_m[-1] < -1e-4)


def test_pso_qaoa_ring_reaches_three_quarters():
    """p = 1 on an 8-ring: <C> = n (1/2 + sin(4 beta) sin(2 gamma) / 4) <= 3n/4
    with E_exact = n, so the approximation ratio approaches 3/4 from below."""
    n = 8
    ring = W.ring_graph(n)
    e_exact = oracle.cut_max(n, ring)[0]
    assert e_exact == n
    f = oracle.qaoa_objective([ring], [n], 1)
    sw, hist, evals = oracle.pso_run(f, 1, 8, 2, rounds=40, seed=2)
    ratio = hist[:, 0] / e_exact
    assert np.all(ratio <= 0.75 + 1e-12) and np.all(np.diff(ratio) >= 0)
    assert ratio[-1] > 0.75 - 1e-4
    assert abs(ratio[0] - evals[0].max() / e_exact) == 0
