"""Pins of the harmonic bias and umbrella integration in the oracle
(oracle/umbrella.py), against closed forms, finite differences and exact
results for a quadratic free energy.

  * V, dV/dxi in closed form, the minimum image across the periodic seam;
  * the force F = -J^T dV/dxi equals -dV/dx by central differences on real
    CVs (a dihedral and a radius of gyration);
  * window mean and covariance from the running sums equal the sample mean
    and (population) covariance;
  * umbrella integration is exact for a quadratic A(xi) = xi^T M xi / 2 +
    b^T xi: the biased mean m solves (M + K) m = K xi0 - b, the mean force
    K (xi0 - m) is grad A(m), and the trapezoidal path integral gives
    A(m_i) - A(m_0) (D = 1 and 2, non-diagonal M);
  * path steps across the periodic seam take the short way.
"""
import numpy as np

from oracle import methods
from oracle.umbrella import Window, harmonic, integrate, wrap

TWO_PI = 2.0 * np.pi


def test_harmonic_closed_form_and_seam():
    V, dV, D = harmonic([0.7, 2.0], [0.2, 1.5], [100.0, 40.0], [True, False])
    assert abs(V - (0.5 * 100.0 * 0.25 + 0.5 * 40.0 * 0.25)) <= 1e-12
    assert np.allclose(dV, [50.0, 20.0], rtol=0, atol=1e-12)
    V, dV, D = harmonic([-np.pi + 0.1], [np.pi - 0.1], [10.0], [True])
    assert abs(D[0] - 0.2) <= 1e-12 and abs(V - 0.5 * 10.0 * 0.04) <= 1e-12
    V2, _, D2 = harmonic([-np.pi + 0.1], [np.pi - 0.1], [10.0], [False])  # not periodic: the long way
    assert abs(D2[0] - (-2 * np.pi + 0.2)) <= 1e-12


def test_force_is_minus_gradient_by_finite_differences():
    from paper_2301_04835_amd import synth

    cvs = [synth.backbone_cvs(4)[0], {"kind": "gyration", "idx": list(range(0, 10))}]
    pos = synth.chain_template(22, 7)
    per = [True, False]
    k = [150.0, 900.0]
    xi, _ = methods.cv_eval(pos, cvs)
    xi0 = xi + np.array([0.4, -0.05])

    def energy(p):
        return harmonic(methods.cv_eval(p, cvs)[0], xi0, k, per)[0]

    xi, J = methods.cv_eval(pos, cvs)
    _, dV, _ = harmonic(xi, xi0, k, per)
    F = methods.chain_rule(-dV, J)
    h = 1e-6
    fd = np.zeros_like(pos)
    for i in range(pos.shape[0]):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fd[i, c] = -(energy(pp) - energy(pm)) / (2 * h)
    assert np.max(np.abs(F - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_window_mean_and_covariance():
    g = np.random.default_rng(3)
    X = g.multivariate_normal([0.3, -0.2, 1.0], [[0.5, 0.1, 0.0], [0.1, 0.2, 0.05], [0.0, 0.05, 0.3]], size=500)
    xi0 = np.array([0.25, -0.1, 0.9])
    w = Window(3)
    for x in X:
        w.add(x - xi0)
    m, C = w.mean_cov(xi0)
    assert w.n == 500
    assert np.allclose(m, X.mean(0), rtol=0, atol=1e-12)
    assert np.allclose(C, np.cov(X.T, bias=True), rtol=0, atol=1e-12)


def _quadratic_case(D, seed):
    g = np.random.default_rng(seed)
    B = g.normal(size=(D, D))
    M = B @ B.T + D * np.eye(D)  # positive definite, not diagonal
    b = g.normal(size=D)
    k = g.uniform(50.0, 200.0, D)
    K = np.diag(k)
    start, end = g.normal(size=D), g.normal(size=D) + 2.0
    xi0s = np.array([start + t * (end - start) for t in np.linspace(0.0, 1.0, 14)])
    means = np.array([np.linalg.solve(M + K, K @ x0 - b) for x0 in xi0s])
    A = lambda x: 0.5 * x @ M @ x + b @ x
    return M, b, k, xi0s, means, A


def test_integration_exact_for_a_quadratic_free_energy():
    for D, seed in ((1, 1), (2, 2), (2, 5)):
        M, b, k, xi0s, means, A = _quadratic_case(D, seed)
        g, Ai = integrate(means, xi0s, k, [False] * D)
        for i in range(len(means)):
            assert np.allclose(g[i], M @ means[i] + b, rtol=0, atol=1e-9)
            assert abs(Ai[i] - (A(means[i]) - A(means[0]))) <= 1e-9 * max(1.0, abs(A(means[i])))


def test_path_across_the_seam_takes_the_short_way():
    means = [[np.pi - 0.2], [-np.pi + 0.2]]
    xi0s = [[np.pi - 0.2 + 0.01], [-np.pi + 0.2 + 0.01]]  # mean force k * 0.01 = 1.0 at both
    g, A = integrate(means, xi0s, [100.0], [True])
    assert np.allclose(g, [[1.0], [1.0]], rtol=0, atol=1e-9)
    assert abs(A[1] - 0.4) <= 1e-9  # not 1.0 * (0.4 - 2 pi)
    assert abs(wrap([TWO_PI + 0.3], [True])[0] - 0.3) <= 1e-12
