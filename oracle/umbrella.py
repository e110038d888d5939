"""Harmonic bias and umbrella integration in FP64 NumPy (test
infrastructure only).

Harmonic biasing (Sec. 2.1.1): the Hamiltonian gains k/2 (xi - xi0)^2
around a point xi0, per CV d with its own k_d > 0.  Umbrella sampling
(Sec. 2.1.2) runs one harmonically biased simulation per point xi0_i of a
path (here: one walker per window); umbrella integration estimates the
mean force at each window and integrates it into the free-energy profile.

Readings where the paper is silent:
  * a periodic CV takes the minimum image of xi - xi0 (period 2 pi);
  * each window keeps the number of samples and the sums of D = xi - xi0
    (minimum image) and of D D^T, so its mean is xi0 + <D> and its
    covariance <D D^T> - <D><D>^T;
  * the mean force on window i, the estimate of dA/dxi at its mean, is
    k (xi0_i - <xi>_i) (the spring force averaged over the window; exact
    when A is quadratic near the window);
  * A along the path: A_0 = 0 and the trapezoidal rule over the straight
    segments between successive window means,
    A_{i+1} = A_i + (g_i + g_{i+1}) . (m_{i+1} - m_i) / 2, with m_i the
    means and g_i the mean forces (differences of periodic means taken with
    the minimum image).
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def wrap(delta, periodic):
    """Minimum image of a difference for the periodic components."""
    d = np.array(delta, dtype=np.float64)
    p = np.asarray(periodic, dtype=bool)
    d[p] -= TWO_PI * np.rint(d[p] / TWO_PI)
    return d


def harmonic(xi, xi0, k, periodic):
    """V = sum_d k_d D_d^2 / 2 and dV/dxi = k D, D = xi - xi0 (wrapped)."""
    D = wrap(np.asarray(xi, dtype=np.float64) - np.asarray(xi0, dtype=np.float64), periodic)
    k = np.asarray(k, dtype=np.float64)
    return 0.5 * float(np.sum(k * D * D)), k * D, D


class Window:
    """Sample count and FP64 sums of D and D D^T of one umbrella window."""

    def __init__(self, D):
        self.n = 0
        self.s1 = np.zeros(D)
        self.s2 = np.zeros((D, D))

    def add(self, Dv):
        self.n += 1
        self.s1 += Dv
        self.s2 += np.outer(Dv, Dv)

    def mean_cov(self, xi0):
        m = self.s1 / self.n
        return np.asarray(xi0, dtype=np.float64) + m, self.s2 / self.n - np.outer(m, m)


def integrate(means, xi0s, k, periodic):
    """Mean forces g_i = k (xi0_i - m_i) and A_i along the path of window
    means (trapezoidal rule, A_0 = 0)."""
    means = np.asarray(means, dtype=np.float64)
    xi0s = np.asarray(xi0s, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    g = k * np.stack([wrap(x0 - m, periodic) for x0, m in zip(xi0s, means)])
    A = np.zeros(len(means))
    for i in range(len(means) - 1):
        step = wrap(means[i + 1] - means[i], periodic)
        A[i + 1] = A[i] + 0.5 * float(np.dot(g[i] + g[i + 1], step))
    return g, A
