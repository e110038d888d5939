"""Pins of the grid-stored bias in the oracle (oracle/grid.py): values the
mathematics fixes, independent of the routine that fills the grid.

  * multilinear read-back reproduces affine node data exactly (weights and
    corner indices, D = 1, 2, 3);
  * one hill on a node: the node holds h and a zero gradient; between two
    nodes along one CV the read-back is the closed-form blend;
  * periodic seam: a cell between the last node and the first reads both,
    with the minimum image; read-back is 2 pi periodic;
  * convergence: the read-back error against the exact hill sum shrinks
    about fourfold when the spacing halves (second order);
  * outside a non-periodic range: zero; at hi: the last node;
  * well-tempered deposits at one node follow the scalar recurrence
    h_k = w exp(-sum_{j<k} h_j / k_B dT).
"""
import numpy as np
import pytest

import oracle
from oracle.grid import BiasGrid, metad_grid_step

TWO_PI = 2.0 * np.pi


@pytest.mark.parametrize("D", [1, 2, 3])
def test_affine_data_reproduced_exactly(D):
    g = np.random.default_rng(D)
    lo = g.uniform(-2, 0, D)
    hi = lo + g.uniform(1, 3, D)
    grid = BiasGrid(lo, hi, [5, 7, 4][:D], [False] * D)
    a = g.normal(size=D)
    A = g.normal(size=(D, D))
    X = grid.nodes()
    grid.V = (X @ a + 0.7).reshape(grid.shape)
    grid.G = (X @ A.T + 1.0).reshape(grid.shape + (D,))
    for _ in range(50):
        x = lo + g.uniform(0, 1, D) * (hi - lo)
        V, G = grid.lookup(x)
        assert abs(V - (x @ a + 0.7)) <= 1e-12
        assert np.max(np.abs(G - (A @ x + 1.0))) <= 1e-12


def test_single_hill_on_a_node_closed_form():
    sigma = [0.35, 0.35]
    grid = BiasGrid([-np.pi, -np.pi], [np.pi, np.pi], [64, 48], [True, True])
    d0, d1 = grid.delta
    i, j = 20, 30
    c = np.array([-np.pi + i * d0, -np.pi + j * d1])
    h = 1.3
    grid.set_hills(c[None], [h], sigma)
    assert abs(grid.V[i, j] - h) <= 1e-15
    assert np.all(np.abs(grid.G[i, j]) <= 1e-15)
    # neighbours along CV 0: h exp(-d0^2 / 2 sigma^2), gradient -(+-d0)/sigma^2 times that
    e = h * np.exp(-d0 * d0 / (2 * sigma[0] ** 2))
    assert abs(grid.V[i + 1, j] - e) <= 1e-15
    assert abs(grid.G[i + 1, j, 0] + d0 / sigma[0] ** 2 * e) <= 1e-14
    # read-back at a fraction t of the way to the next node along CV 0
    for t in (0.0, 0.25, 0.5, 0.9):
        V, G = grid.lookup(c + np.array([t * d0, 0.0]))
        assert abs(V - ((1 - t) * h + t * e)) <= 1e-14
        assert abs(G[0] - t * (-d0 / sigma[0] ** 2 * e)) <= 1e-13
        assert abs(G[1]) <= 1e-15


def test_periodic_seam_and_period():
    sigma = [0.3]
    grid = BiasGrid([-np.pi], [np.pi], [40], [True])
    d = grid.delta[0]
    c = np.pi - 0.25 * d  # between the last node (pi - d) and the first (-pi = pi)
    grid.set_hills([[c]], [1.0], sigma)
    last = np.exp(-(0.75 * d) ** 2 / (2 * sigma[0] ** 2))
    first = np.exp(-(0.25 * d) ** 2 / (2 * sigma[0] ** 2))  # minimum image across the seam
    assert abs(grid.V[-1] - last) <= 1e-15 and abs(grid.V[0] - first) <= 1e-15
    x = np.pi - 0.4 * d  # in the seam cell, weight 0.6 on node 0
    V, _ = grid.lookup([x])
    assert abs(V - (0.4 * last + 0.6 * first)) <= 1e-14
    for x in np.linspace(-3, 3, 13):
        assert abs(grid.lookup([x])[0] - grid.lookup([x + TWO_PI])[0]) <= 1e-12
        assert abs(grid.lookup([x])[0] - grid.lookup([x - TWO_PI])[0]) <= 1e-12


def test_second_order_convergence_to_the_hill_sum():
    g = np.random.default_rng(5)
    K = 40
    C = g.uniform(-np.pi, np.pi, size=(K, 2))
    H = g.uniform(0.5, 1.5, size=K)
    sigma = [0.35, 0.35]
    per = [TWO_PI, TWO_PI]
    X = g.uniform(-np.pi, np.pi, size=(200, 2))
    ref = [oracle.hillsum(x, C, H, sigma, per) for x in X]
    errs = []
    for n in (64, 128, 256, 512):
        grid = BiasGrid([-np.pi, -np.pi], [np.pi, np.pi], [n, n], [True, True])
        grid.set_hills(C, H, sigma)
        eV, eG = [], []
        for x, (Vr, Gr) in zip(X, ref):
            V, G = grid.lookup(x)
            eV.append(V - Vr)
            eG.extend(G - Gr)
        errs.append((np.sqrt(np.mean(np.square(eV))), np.sqrt(np.mean(np.square(eG)))))
    for k in range(3):  # rms errors over the sample points
        assert 3.3 <= errs[k][0] / errs[k + 1][0] <= 4.8
        assert 3.3 <= errs[k][1] / errs[k + 1][1] <= 4.8


def test_outside_a_nonperiodic_range():
    grid = BiasGrid([1.0], [2.0], [10], [False])
    assert grid.shape == (11,)
    grid.V[:] = np.arange(11.0)
    for x in (0.999, 2.001):
        V, G = grid.lookup([x])
        assert V == 0.0 and np.all(G == 0.0)
    assert abs(grid.lookup([2.0])[0] - 10.0) <= 1e-12  # hi is the last node
    assert abs(grid.lookup([1.0])[0] - 0.0) <= 1e-12
    assert abs(grid.lookup([1.55])[0] - 5.5) <= 1e-12


def test_well_tempered_deposits_at_a_node():
    """Hills deposited one after another at a node: the node value is the
    sum of the heights so far, so h_k = w exp(-sum_{j<k} h_j / k_B dT)."""
    w, kdT = 1.2, oracle.KB * 300.0 * 5.0
    sigma = [0.35, 0.35]
    grid = BiasGrid([-np.pi, -np.pi], [np.pi, np.pi], [32, 32], [True, True])
    s = np.array([-np.pi + 5 * grid.delta[0], -np.pi + 9 * grid.delta[1]])
    C, H = [], []
    total = 0.0
    for k in range(30):
        V, _ = grid.lookup(s)
        assert abs(V - total) <= 1e-12 * max(1.0, total)
        h = oracle.wt_height(w, V, kdT)
        assert abs(h - w * np.exp(-total / kdT)) <= 1e-14
        total += h
        C.append(s)
        H.append(h)
        grid.set_hills(np.array(C), np.array(H), sigma)


def test_grid_step_force_is_the_chain_rule_of_the_read_back():
    """metad_grid_step: F = -J^T dV/dxi with dV/dxi the read-back at xi, and
    the deposit's height from the read-back V."""
    from paper_2301_04835_amd import synth

    cvs = synth.backbone_cvs(4)
    pos = synth.chain_template(22, 1)
    xi, J = oracle.methods.cv_eval(pos, cvs)
    grid = BiasGrid([-np.pi, -np.pi], [np.pi, np.pi], [50, 50], [True, True])
    C = np.random.default_rng(2).uniform(-np.pi, np.pi, size=(30, 2))
    grid.set_hills(C, np.ones(30), [0.35, 0.35])
    r = metad_grid_step(pos, cvs, grid, 1.2, 6.0, 500, 0)
    V, G = grid.lookup(xi)
    assert r["V"] == V
    assert np.allclose(r["F"], -np.einsum("d,dni->ni", G, J), rtol=0, atol=1e-14)
    assert r["deposit"] is not None and r["deposit"][1] == oracle.wt_height(1.2, V, 6.0)
