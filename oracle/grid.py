"""Grid-stored metadynamics bias in FP64 NumPy (test infrastructure only).

The paper lets metadynamics keep its bias on a pre-defined grid instead of
summing every hill at every step, trading accuracy for speed (Sec. 2.1.5,
the closing remark on optional grid storage).  It fixes neither the grid
nor how a value is read back; the readings taken here:

  * nodes: per CV d, spacing delta_d = (hi_d - lo_d) / n_d; a periodic CV
    (its range must be one period) has the n_d nodes lo_d + i delta_d,
    i < n_d, and wraps; a non-periodic CV has the n_d + 1 nodes up to and
    including hi_d.  Row-major, first CV slowest.
  * stored values: the bias of the hill list at every node and its gradient
    dV/dxi there (the exact hill sum of Sec. 2.1.5 evaluated at the node).
  * read-back: multilinear interpolation of V and of each component of
    dV/dxi over the 2^D nodes of the cell holding xi (the force uses the
    interpolated gradient, not the derivative of the interpolated V).
  * outside the range of a non-periodic CV: no bias (V = 0, dV/dxi = 0) and
    no deposit.
  * well-tempered height: w exp(-V(s) / k_B dT) with V(s) the bias the step
    read from the grid.
"""
import numpy as np

from . import _clib


class BiasGrid:
    """V and dV/dxi of a hill list stored at the nodes of a regular grid."""

    def __init__(self, lo, hi, nbins, periodic):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.n = [int(k) for k in nbins]
        self.periodic = [bool(p) for p in periodic]
        self.D = len(self.n)
        self.delta = (self.hi - self.lo) / np.asarray(self.n, dtype=np.float64)
        self.shape = tuple(k if p else k + 1 for k, p in zip(self.n, self.periodic))
        self.V = np.zeros(self.shape)
        self.G = np.zeros(self.shape + (self.D,))

    def nodes(self):
        """Coordinates of every node, (prod(shape), D), row-major."""
        axes = [self.lo[d] + self.delta[d] * np.arange(self.shape[d]) for d in range(self.D)]
        mesh = np.meshgrid(*axes, indexing="ij")
        return np.stack([m.reshape(-1) for m in mesh], axis=1)

    def set_hills(self, centers, heights, sigma):
        """Store the exact bias of the hill list (centres K x D, heights K)
        and its gradient at every node."""
        period = np.where(self.periodic, self.hi - self.lo, 0.0)
        X = self.nodes()
        if len(heights) == 0:
            self.V[...] = 0.0
            self.G[...] = 0.0
            return
        V, dV = _clib.hillsum_batch(X, None, np.asarray(centers, dtype=np.float64).reshape(-1, self.D),
                                    np.asarray(heights, dtype=np.float64), sigma, period)
        self.V = V.reshape(self.shape)
        self.G = dV.reshape(self.shape + (self.D,))

    def corners(self, xi):
        """The cell of xi: per CV (i0, i1, t) with the interpolation weight t
        of node i1, or None outside a non-periodic range."""
        out = []
        for d in range(self.D):
            u = (xi[d] - self.lo[d]) / self.delta[d]
            i0 = int(np.floor(u))
            t = u - i0
            if self.periodic[d]:
                i0 %= self.n[d]
                out.append((i0, (i0 + 1) % self.n[d], t))
            else:
                if u < 0.0 or u > self.n[d]:
                    return None
                if i0 == self.n[d]:  # xi == hi: the last cell, t = 1
                    i0, t = self.n[d] - 1, 1.0
                out.append((i0, i0 + 1, t))
        return out

    def lookup(self, xi):
        """(V, dV/dxi) at xi by multilinear interpolation (zero outside)."""
        c = self.corners(np.asarray(xi, dtype=np.float64))
        if c is None:
            return 0.0, np.zeros(self.D)
        V = 0.0
        G = np.zeros(self.D)
        for corner in range(1 << self.D):
            idx = []
            wgt = 1.0
            for d in range(self.D):
                i0, i1, t = c[d]
                if (corner >> (self.D - 1 - d)) & 1:
                    idx.append(i1)
                    wgt *= t
                else:
                    idx.append(i0)
                    wgt *= 1.0 - t
            V += wgt * self.V[tuple(idx)]
            G += wgt * self.G[tuple(idx)]
        return V, G


def metad_grid_step(pos, cvs, grid, w, kdT, stride, step, box=None):
    """One step of metadynamics with the bias read from a grid: the force
    -sum_d dV/dxi_d dxi_d/dx from the interpolated gradient; when
    t mod stride == 0 and xi lies on the grid, a hill at s = xi with height
    w exp(-V(s)/k_B dT) (V read from the grid) to be added to the list."""
    from .methods import cv_eval, chain_rule

    xi, J = cv_eval(pos, cvs, box)
    V, dV = grid.lookup(xi)
    F = chain_rule(-dV, J)
    dep = None
    if stride > 0 and step % stride == 0 and grid.corners(xi) is not None:
        dep = (xi.copy(), _clib.wt_height(w, V, kdT))
    return {"xi": xi, "J": J, "V": V, "dV": dV, "F": F, "deposit": dep}
