"""Composition of one biasing step in FP64 NumPy (test infrastructure only).

Follows Sec. 2 of the paper: collective variables xi(x) and their gradients
(obtained in PySAGES by automatic differentiation, here by the analytic
gradients of ``oracle.c``), the metadynamics / well-tempered metadynamics
bias (Sec. 2.1.5) and the adaptive biasing force (Sec. 2.1.4), and the
biasing force that is added to the engine's net forces (Sec. 2, the
force-like callback).
"""
import numpy as np

from . import _clib

TWO_PI = 2.0 * np.pi


def cv_periods(cvs):
    """Period of each CV: 2 pi for dihedral angles, 0 (not periodic) otherwise."""
    return np.array([TWO_PI if c["kind"] == "dihedral" else 0.0 for c in cvs], dtype=np.float64)


def cv_eval(pos, cvs, box=None):
    """xi (D,) and the dense Jacobian J (D, natoms, 3) of a list of CVs.

    cvs: list of dicts, one per CV:
      {"kind": "dihedral", "idx": [i, j, k, l]}
      {"kind": "gyration", "idx": [...]}
      {"kind": "coordination", "a": [...], "b": [...], "r0": r0, "n": n, "m": m,
       "rcut": rcut (0: all pairs), "normalize": bool}
    Dihedrals and the radius of gyration use positions as given (molecules
    unwrapped); the coordination number uses the minimum image in ``box``.
    """
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    D = len(cvs)
    xi = np.zeros(D)
    J = np.zeros((D, pos.shape[0], 3))
    for d, c in enumerate(cvs):
        k = c["kind"]
        if k == "dihedral":
            idx = np.asarray(c["idx"], dtype=np.int64)
            phi, g = _clib.dihedral(pos[idx])
            xi[d] = phi
            for s in range(4):
                J[d, idx[s]] += g[s]
        elif k == "gyration":
            idx = np.asarray(c["idx"], dtype=np.int64)
            rg, g = _clib.gyration(pos[idx])
            xi[d] = rg
            np.add.at(J[d], idx, g)
        elif k == "coordination":
            cn, g = _clib.coordination(pos, c["a"], c["b"], c["r0"], c["n"], c["m"], c.get("rcut", 0.0),
                                       box, c.get("normalize", False))
            xi[d] = cn
            J[d] = g
        else:
            raise ValueError("unknown CV kind %r" % (k,))
    return xi, J


def chain_rule(coef, J):
    """Per-atom force sum_d coef_d J_d (J: D x natoms x 3)."""
    return np.einsum("d,dni->ni", np.asarray(coef, dtype=np.float64), J)


def metad_step(pos, cvs, centers, heights, sigma, w, kdT, stride, step, box=None):
    """One metadynamics / well-tempered metadynamics step (Sec. 2.1.5).

    The bias at step t is the sum of the hills deposited before t.  The force
    F = -sum_d dV/dxi_d dxi_d/dx is returned for every atom.  When
    t mod stride == 0 (t = 0 included) a hill is deposited at s = xi(x_t) with
    height w exp(-V_t(s)/(k_B dT)) (plain metadynamics: kdT <= 0, height w).
    """
    xi, J = cv_eval(pos, cvs, box)
    per = cv_periods(cvs)
    if len(heights):
        V, dV = _clib.hillsum(xi, centers, heights, sigma, per)
    else:
        V, dV = 0.0, np.zeros(len(cvs))
    F = chain_rule(-dV, J)
    dep = None
    if stride > 0 and step % stride == 0:
        dep = (xi.copy(), _clib.wt_height(w, V, kdT))
    return {"xi": xi, "J": J, "V": V, "dV": dV, "F": F, "deposit": dep}


# ------------------------------------------------------------------------- #
# Adaptive biasing force (Sec. 2.1.4; Darve et al. 2008; threshold N from   #
# the parameter table of the appendix).                                     #
# ------------------------------------------------------------------------- #
def abf_bin(xi, lo, hi, nbins, periodic):
    """Row-major bin index of xi on the grid [lo, hi) with nbins per CV.

    Periodic CVs wrap the per-CV index modulo nbins; a non-periodic CV
    outside [lo, hi) gives -1 (the sample is dropped and gets no bias).
    """
    k = 0
    for d in range(len(xi)):
        delta = (hi[d] - lo[d]) / nbins[d]
        i = int(np.floor((xi[d] - lo[d]) / delta))
        if periodic[d]:
            i %= nbins[d]
        elif i < 0 or i >= nbins[d]:
            return -1
        k = k * nbins[d] + i
    return k


def abf_theta(J, Fsys):
    """Instantaneous estimate of dA/dxi from the projected system force:
    theta = -(J J^T)^{-1} J F  (unit masses; J: D x natoms x 3)."""
    Jm = J.reshape(J.shape[0], -1)
    G = Jm @ Jm.T
    return -np.linalg.solve(G, Jm @ np.asarray(Fsys, dtype=np.float64).reshape(-1))


class AbfGrid:
    """Histogram N and force sums Fsum of an ABF run (FP64 sums)."""

    def __init__(self, lo, hi, nbins, periodic, n_threshold):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.nbins = [int(n) for n in nbins]
        self.periodic = [bool(p) for p in periodic]
        self.n_threshold = int(n_threshold)
        nb = int(np.prod(self.nbins))
        self.N = np.zeros(nb, dtype=np.int64)
        self.Fsum = np.zeros((nb, len(self.nbins)))


def abf_step(grid, xi, J, Fsys):
    """One ABF step: bias b = Fsum[k] / max(N[k], N_thr) from the samples
    before this step, then N[k] += 1 and Fsum[k] += theta.  Returns
    (b, per-atom biasing force sum_d b_d J_d, bin index, theta)."""
    D = len(xi)
    k = abf_bin(xi, grid.lo, grid.hi, grid.nbins, grid.periodic)
    theta = abf_theta(J, Fsys)
    if k < 0:
        b = np.zeros(D)
    else:
        den = max(int(grid.N[k]), grid.n_threshold)
        b = grid.Fsum[k] / den if den > 0 else np.zeros(D)
        grid.N[k] += 1
        grid.Fsum[k] += theta
    return b, chain_rule(b, J), k, theta


# ------------------------------------------------------------------------- #
# ABF with the momentum-derivative estimator (Darve et al. 2008, the         #
# algorithm the paper's ABF follows, Sec. 2.1.4).  Reading: with masses M,   #
# the CV-space momentum is W p = (J M^-1 J^T)^-1 J M^-1 p; over a step of    #
# length dt it changes by the system's generalised force plus the bias b     #
# applied during that step, so                                              #
#   theta_t = b_{t-1} - ((W p)_t - (W p)_{t-1}) / dt                         #
# estimates dA/dxi (backward difference, binned at the current xi); the      #
# first step only records (W p)_0 and b_0.                                   #
# ------------------------------------------------------------------------- #
def abf_momentum_wp(J, p, inv_mass):
    """W p = (J M^-1 J^T)^-1 J M^-1 p (J: D x natoms x 3, p: natoms x 3,
    inv_mass: natoms)."""
    Jm = J * np.asarray(inv_mass, dtype=np.float64)[None, :, None]
    G = Jm.reshape(J.shape[0], -1) @ J.reshape(J.shape[0], -1).T
    u = Jm.reshape(J.shape[0], -1) @ np.asarray(p, dtype=np.float64).reshape(-1)
    return np.linalg.solve(G, u)


def abf_step_momentum(grid, xi, J, p, inv_mass, dt, prev):
    """One ABF step with the momentum estimator.  prev: (W p, b) of the
    previous step or None.  Returns (b, per-atom biasing force, bin, theta
    or None, (W p, b) for the next step)."""
    D = len(xi)
    k = abf_bin(xi, grid.lo, grid.hi, grid.nbins, grid.periodic)
    wp = abf_momentum_wp(J, p, inv_mass)
    theta = None if prev is None else prev[1] - (wp - prev[0]) / dt
    if k < 0:
        b = np.zeros(D)
    else:
        den = max(int(grid.N[k]), grid.n_threshold)
        b = grid.Fsum[k] / den if den > 0 else np.zeros(D)
        if theta is not None:
            grid.N[k] += 1
            grid.Fsum[k] += theta
    return b, chain_rule(b, J), k, theta, (wp, b)
