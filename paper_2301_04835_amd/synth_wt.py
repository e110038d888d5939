"""Seeded hill list shaped like a converged well-tempered run (input recipe).

The surrogate workload needs the bias of a long well-tempered metadynamics
run on two periodic CVs: 100,000 hills of width 0.3 rad whose heights start
from w ~ U[0.5, 1.5] kJ/mol and are tempered by the bias already deposited
(Sec. 2.1.5).  Hills with uniformly random centres would give a rough field
that no small network could follow; a real run deposits along trajectories
that the growing bias pushes out of the filled regions.  This recipe plays
such a run out cheaply:

  * W walkers move by overdamped Langevin dynamics (Euler-Maruyama) on an
    analytic periodic free-energy surface F(phi, psi) plus the bias;
  * every `stride` steps each walker drops a hill at its position with
    height w_k exp(-Vg / (k_B dT)), w_k ~ U[0.5, 1.5];
  * the bias that steers the walkers and tempers the heights, Vg, is the
    recipe's own coarse estimate: the Gaussians are summed onto a 256 x 256
    periodic grid (separable, one outer product per deposition round) and
    read back by bilinear interpolation.

Only the hill list (centres, heights) leaves this module.  The grid
estimate is used by neither the CPU oracle nor the library: each computes
the bias of the list on its own, so the recipe cannot hide a mistake in
either.
"""
import numpy as np

KB = 0.008314462618  # kJ/(mol K)
TWO_PI = 2.0 * np.pi


def fes(phi, psi):
    """Analytic periodic free-energy surface (kJ/mol): a few low Fourier
    modes with basins and barriers of a few tens of kJ/mol."""
    return (-12.0 * np.cos(phi - 1.0) - 8.0 * np.cos(psi + 2.0) - 6.0 * np.cos(phi + psi - 0.5)
            + 4.0 * np.cos(2.0 * phi - psi + 1.0))


def fes_grad(phi, psi):
    gp = 12.0 * np.sin(phi - 1.0) + 6.0 * np.sin(phi + psi - 0.5) - 8.0 * np.sin(2.0 * phi - psi + 1.0)
    gs = 8.0 * np.sin(psi + 2.0) + 6.0 * np.sin(phi + psi - 0.5) + 4.0 * np.sin(2.0 * phi - psi + 1.0)
    return gp, gs


def wt_hills(K=100000, sigma=0.3, w_range=(0.5, 1.5), temperature=300.0, bias_factor=6.0, n_walkers=64,
             stride=10, step=0.03, grid=256, seed=41):
    """Hill list (centres float32 K x 2 in [-pi, pi), heights float32 K) of
    the multiple-walker run described in the module docstring.  `step` is
    the rms Brownian displacement per step (rad); K is rounded down to a
    multiple of n_walkers."""
    g = np.random.default_rng(seed)
    kT = KB * temperature
    kdT = KB * temperature * (bias_factor - 1.0)
    x = g.uniform(-np.pi, np.pi, size=(n_walkers, 2))
    vg = np.zeros((grid, grid))
    hg = TWO_PI / grid
    ax = -np.pi + hg * np.arange(grid)
    mob = 0.5 * step * step / kT  # D dt / kT
    rounds = K // n_walkers
    C = np.empty((rounds * n_walkers, 2))
    H = np.empty(rounds * n_walkers)

    def bilinear(p):
        u = (p + np.pi) / hg
        i0 = np.floor(u).astype(np.int64)
        f = u - i0
        i0 %= grid
        i1 = (i0 + 1) % grid
        v00 = vg[i0[:, 0], i0[:, 1]]
        v10 = vg[i1[:, 0], i0[:, 1]]
        v01 = vg[i0[:, 0], i1[:, 1]]
        v11 = vg[i1[:, 0], i1[:, 1]]
        fx, fy = f[:, 0], f[:, 1]
        val = (1 - fx) * (1 - fy) * v00 + fx * (1 - fy) * v10 + (1 - fx) * fy * v01 + fx * fy * v11
        gx = ((1 - fy) * (v10 - v00) + fy * (v11 - v01)) / hg
        gy = ((1 - fx) * (v01 - v00) + fx * (v11 - v10)) / hg
        return val, gx, gy

    for r in range(rounds):
        for _ in range(stride):
            _, bx, by = bilinear(x)
            fx, fy = fes_grad(x[:, 0], x[:, 1])
            x[:, 0] += -mob * (fx + bx) + step * g.normal(size=n_walkers)
            x[:, 1] += -mob * (fy + by) + step * g.normal(size=n_walkers)
            x = (x + np.pi) % TWO_PI - np.pi
        vd, _, _ = bilinear(x)
        h = g.uniform(w_range[0], w_range[1], size=n_walkers) * np.exp(-vd / kdT)
        C[r * n_walkers:(r + 1) * n_walkers] = x
        H[r * n_walkers:(r + 1) * n_walkers] = h
        dx = ax[None, :] - x[:, 0:1]
        dx -= TWO_PI * np.rint(dx / TWO_PI)
        dy = ax[None, :] - x[:, 1:2]
        dy -= TWO_PI * np.rint(dy / TWO_PI)
        vg += (np.exp(-dx * dx / (2 * sigma * sigma)) * h[:, None]).T @ np.exp(-dy * dy / (2 * sigma * sigma))
    C32 = C.astype(np.float32)
    # float32 rounding can land exactly on +pi; keep centres in [-pi, pi)
    C32[C32 >= np.float32(np.pi)] -= np.float32(TWO_PI)
    return C32, H.astype(np.float32)


def torus_points(n, seed):
    """n points uniform on [-pi, pi)^2 (training and test samples)."""
    return np.random.default_rng(seed).uniform(-np.pi, np.pi, size=(n, 2))
