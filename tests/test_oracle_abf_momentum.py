"""Pins of the ABF momentum-derivative estimator in the oracle
(oracle.methods.abf_step_momentum, abf_momentum_wp).

  * W J^T = identity (a generalised force maps to itself) on real CVs;
  * two atoms and xi = x_0 - x_1: W p = mu (v_0 - v_1) with the reduced
    mass mu (the textbook generalised momentum; catches M for M^-1);
  * linear CVs with arbitrary masses under the force -J^T grad A(xi) of a
    quadratic A plus the ABF bias, stepped by symplectic Euler: every
    estimate equals grad A at the step's start exactly;
  * the first step records and adds no sample.
"""
import numpy as np

import oracle
from oracle.methods import AbfGrid, abf_momentum_wp, abf_step_momentum, cv_eval


def test_w_maps_generalised_forces_to_themselves():
    from paper_2301_04835_amd import synth

    cvs = [synth.backbone_cvs(4)[0], {"kind": "gyration", "idx": list(range(0, 12))}]
    pos = synth.chain_template(22, 3)
    _, J = cv_eval(pos, cvs)
    inv_m = 1.0 / np.random.default_rng(1).uniform(1.0, 16.0, 22)
    c = np.array([0.7, -2.5])
    p = np.einsum("d,dni->ni", c, J)
    assert np.allclose(abf_momentum_wp(J, p, inv_m), c, rtol=0, atol=1e-10)


def test_reduced_mass_momentum():
    J = np.zeros((1, 2, 3))
    J[0, 0, 0], J[0, 1, 0] = 1.0, -1.0
    m0, m1 = 2.0, 7.0
    v0, v1 = 0.3, -0.45
    p = np.array([[m0 * v0, 5.0, 1.0], [m1 * v1, -2.0, 0.5]])  # y, z momenta do not enter
    mu = m0 * m1 / (m0 + m1)
    assert abs(abf_momentum_wp(J, p, [1 / m0, 1 / m1])[0] - mu * (v0 - v1)) <= 1e-14


def test_linear_cvs_recover_the_mean_force_exactly():
    """xi = (x_0 - x_1, y_2) for three atoms of masses 1.5, 4, 12; A(xi) =
    xi^T Q xi / 2 + c^T xi; F = -J^T grad A(xi(x_t)) + J^T b_t; p_{t+1} =
    p_t + F dt, x_{t+1} = x_t + M^-1 p_{t+1} dt."""
    J = np.zeros((2, 3, 3))
    J[0, 0, 0], J[0, 1, 0], J[1, 2, 1] = 1.0, -1.0, 1.0
    m = np.array([1.5, 4.0, 12.0])
    Q = np.array([[3.0, 0.4], [0.4, 1.5]])
    cvec = np.array([0.2, -0.7])
    xi_of = lambda x: np.array([x[0, 0] - x[1, 0], x[2, 1]])
    gradA = lambda s: Q @ s + cvec
    grid = AbfGrid([-3.0, -3.0], [3.0, 3.0], [12, 12], [False, False], 3)
    g = np.random.default_rng(2)
    x = g.normal(scale=0.3, size=(3, 3))
    p = g.normal(size=(3, 3))
    dt = 0.01
    prev = None
    for t in range(200):
        s = xi_of(x)
        b, Fb, k, theta, prev_new = abf_step_momentum(grid, s, J, p, 1.0 / m, dt, prev)
        if t == 0:
            assert theta is None and grid.N.sum() == 0
        else:
            assert np.allclose(theta, gradA(s_prev), rtol=0, atol=1e-9)
        F = -np.einsum("d,dni->ni", gradA(s), J) + Fb
        p = p + F * dt
        x = x + p / m[:, None] * dt
        prev, s_prev = prev_new, s
    assert grid.N.sum() == 199
