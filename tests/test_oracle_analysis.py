"""Pins of the free-energy analysis in the oracle (oracle/analysis.py).

  * metadynamics: one hill gives F = -gamma/(gamma - 1) h exp(-D^2/2s^2)
    shifted to min 0 (well-tempered), the plain factor is 1;
  * ABF integration is exact for a quadratic A sampled at the bin centres
    (D = 1, 2, a non-diagonal form, a hole of unvisited bins), equals the
    trapezoidal rule in 1-D, and converges at second order for a periodic
    A on a periodic grid; unvisited bins stay NaN.
"""
import numpy as np

import oracle
from oracle.analysis import abf_fes, grid_nodes, metad_fes

TWO_PI = 2.0 * np.pi


def test_metad_fes_single_hill_factors():
    sigma = [0.3, 0.4]
    c = np.array([[0.5, -1.0]])
    h = np.array([2.0])
    lo, hi, nb, per = [-np.pi, -np.pi], [np.pi, np.pi], [24, 30], [True, True]
    X, shape = grid_nodes(lo, hi, nb, per)
    D = X - c
    D -= TWO_PI * np.rint(D / TWO_PI)
    g = h[0] * np.exp(-D[:, 0] ** 2 / (2 * sigma[0] ** 2) - D[:, 1] ** 2 / (2 * sigma[1] ** 2))
    T, gamma = 300.0, 6.0
    kdT = oracle.KB * T * (gamma - 1)
    F = metad_fes(c, h, sigma, [TWO_PI, TWO_PI], lo, hi, nb, per, T, kdT)
    ref = -gamma / (gamma - 1) * g
    assert F.shape == (24, 30)
    assert np.max(np.abs(F.reshape(-1) - (ref - ref.min()))) <= 1e-12
    Fp = metad_fes(c, h, sigma, [TWO_PI, TWO_PI], lo, hi, nb, per, T, 0.0)
    assert np.max(np.abs(Fp.reshape(-1) - (-g + g.max()))) <= 1e-12


def _abf_from_gradient(grad, nbins, lo, delta, counts=None):
    D = len(nbins)
    centres = [lo[d] + (np.arange(nbins[d]) + 0.5) * delta[d] for d in range(D)]
    mesh = np.meshgrid(*centres, indexing="ij")
    X = np.stack([m.reshape(-1) for m in mesh], 1)
    G = np.array([grad(x) for x in X])
    N = np.ones(len(X), dtype=np.int64) if counts is None else counts
    return N, G * N[:, None], X


def test_abf_exact_for_quadratic_2d_with_hole():
    M = np.array([[2.0, 0.7], [0.7, 1.2]])
    b = np.array([0.3, -0.5])
    A = lambda x: 0.5 * x @ M @ x + b @ x
    nb, lo, delta = [12, 9], [-1.0, -2.0], [0.25, 0.4]
    counts = np.random.default_rng(1).integers(1, 50, size=12 * 9)
    counts.reshape(12, 9)[5:7, 3:5] = 0  # a hole
    N, Fs, X = _abf_from_gradient(lambda x: M @ x + b, nb, lo, delta, counts)
    Ar = abf_fes(N, Fs, nb, delta, [False, False])
    exact = np.array([A(x) for x in X]).reshape(12, 9)
    vis = counts.reshape(12, 9) > 0
    assert np.all(np.isnan(Ar[~vis]))
    e = exact[vis] - exact[vis].min()
    assert np.max(np.abs(Ar[vis] - e)) <= 1e-10


def test_abf_1d_is_the_trapezoidal_rule():
    nb, lo, delta = [20], [0.0], [0.1]
    g = np.random.default_rng(2).normal(size=20)
    N = np.full(20, 3)
    Ar = abf_fes(N, (g * 3)[:, None], nb, delta, [False])
    trap = np.concatenate([[0.0], np.cumsum(0.5 * (g[:-1] + g[1:]) * 0.1)])
    assert np.max(np.abs(Ar - (trap - trap.min()))) <= 1e-12


def test_abf_periodic_second_order():
    A = lambda x: np.cos(x[0]) + 0.5 * np.sin(2 * x[1])
    grad = lambda x: np.array([-np.sin(x[0]), np.cos(2 * x[1])])
    errs = []
    for n in (16, 32, 64):
        nb, lo, delta = [n, n], [-np.pi, -np.pi], [TWO_PI / n, TWO_PI / n]
        N, Fs, X = _abf_from_gradient(grad, nb, lo, delta)
        Ar = abf_fes(N, Fs, nb, delta, [True, True]).reshape(-1)
        exact = np.array([A(x) for x in X])
        exact -= exact.min()
        errs.append(np.max(np.abs((Ar - Ar.mean()) - (exact - exact.mean()))))
    assert 3.3 <= errs[0] / errs[1] <= 4.7 and 3.3 <= errs[1] / errs[2] <= 4.7
