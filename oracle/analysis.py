"""Free energies from a finished run, in FP64 NumPy (test infrastructure
only): the analysis step that closes the loop from a bias to a free-energy
surface (Sec. 2, the analysis of a run's state).

Metadynamics (Sec. 2.1.5): the deposited bias V estimates the free energy
as F = -V (plain) or, well-tempered, F = -(T + dT)/dT V (the bias converges
to -(dT/(T + dT)) F); evaluated at the nodes of an analysis grid and shifted
so that min F = 0.

ABF (Sec. 2.1.4): the grid of running mean forces g = Fsum / N estimates
dA/dxi at the bin centres.  Reading for D >= 1: A minimises
  sum over pairs (i, j) of neighbouring visited bins along CV d of
      ((A_j - A_i) / delta_d - (g_i,d + g_j,d) / 2)^2
(periodic CVs wrap), solved here by dense least squares; in 1-D this is the
trapezoidal rule, and it is exact for a quadratic A.  Unvisited bins are
left out (NaN); the visited ones are shifted so that min A = 0 (one
connected set of visited bins is assumed).
"""
import numpy as np

from . import _clib

KB = _clib.KB


def grid_nodes(lo, hi, nbins, periodic):
    """Analysis-grid nodes (row-major, first CV slowest): nbins per periodic
    CV, nbins + 1 up to hi otherwise."""
    axes = []
    for l, h, n, p in zip(lo, hi, nbins, periodic):
        d = (h - l) / n
        axes.append(l + d * np.arange(n if p else n + 1))
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1), tuple(len(a) for a in axes)


def metad_fes(centers, heights, sigma, period, lo, hi, nbins, periodic, temperature, kdT):
    """F at the nodes of the analysis grid (shape of the grid)."""
    X, shape = grid_nodes(lo, hi, nbins, periodic)
    V, _ = _clib.hillsum_batch(X, None, np.asarray(centers, dtype=np.float64), np.asarray(heights, dtype=np.float64),
                               sigma, period)
    factor = (KB * temperature + kdT) / kdT if kdT > 0 else 1.0
    F = -factor * V
    return (F - F.min()).reshape(shape)


def abf_fes(N, Fsum, nbins, delta, periodic):
    """A at the bin centres from the ABF counts N (bins) and sums Fsum
    (bins x D): least squares over the edges between visited bins."""
    nbins = [int(n) for n in nbins]
    D = len(nbins)
    nb = int(np.prod(nbins))
    N = np.asarray(N).reshape(nb)
    g = np.asarray(Fsum, dtype=np.float64).reshape(nb, D) / np.maximum(N, 1)[:, None]
    vis = N > 0
    idx = np.full(nb, -1)
    idx[vis] = np.arange(int(vis.sum()))
    rows, rhs = [], []
    strides = [int(np.prod(nbins[d + 1:])) for d in range(D)]
    for b in range(nb):
        if not vis[b]:
            continue
        coord = [(b // strides[d]) % nbins[d] for d in range(D)]
        for d in range(D):
            c = coord[d] + 1
            if c == nbins[d]:
                if not periodic[d]:
                    continue
                c = 0
            nbr = b + (c - coord[d]) * strides[d]
            if not vis[nbr]:
                continue
            r = np.zeros(int(vis.sum()))
            r[idx[nbr]] += 1.0 / delta[d]
            r[idx[b]] -= 1.0 / delta[d]
            rows.append(r)
            rhs.append(0.5 * (g[b, d] + g[nbr, d]))
    A = np.full(nb, np.nan)
    if rows:
        sol = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
        A[vis] = sol - sol.min()
    elif vis.any():
        A[vis] = 0.0
    return A.reshape(nbins)
