"""Pins of the FP64 oracle's collective variables against closed forms,
invariants, finite differences and brute force (no GPU).

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

import oracle

rng = np.random.default_rng(12345)


def central_fd(f, x, h):
    x = np.array(x, dtype=np.float64)
    g = np.zeros_like(x)
    for i in np.ndindex(x.shape):
        xp = x.copy()
        xm = x.copy()
        xp[i] += h
        xm[i] -= h
        g[i] = (f(xp) - f(xm)) / (2 * h)
    return g


def rot(a, b, c):
    ca, sa, cb, sb, cc, sc = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)
    Rz = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1]])
    Ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    Rx = np.array([[1, 0, 0], [0, cc, -sc], [0, sc, cc]])
    return Rz @ Ry @ Rx


# --------------------------------------------------------------------- O1
@pytest.mark.parametrize("theta", [0.0, 0.3, 1.0, np.pi / 2, 2.5, -0.7, -2.9, np.pi - 1e-9, -np.pi + 1e-9])
def test_dihedral_constructed_angle(theta):
    # r1 on +x, axis along +z, r4 rotated by theta about the axis => phi = theta
    r = [[1, 0, 0], [0, 0, 0], [0, 0, 1], [np.cos(theta), np.sin(theta), 1]]
    phi, _ = oracle.dihedral(r)
    assert abs(phi - theta) < 1e-12


def _projection_dihedral(r):
    """Independent definition: angle between the projections of r1-r2 and
    r4-r3 on the plane normal to the axis r3-r2, signed by the axis."""
    r = np.asarray(r, dtype=np.float64)
    ax = r[2] - r[1]
    ax /= np.linalg.norm(ax)
    u = (r[0] - r[1]) - np.dot(r[0] - r[1], ax) * ax
    v = (r[3] - r[2]) - np.dot(r[3] - r[2], ax) * ax
    return math.atan2(np.dot(np.cross(u, v), ax), np.dot(u, v))


def test_dihedral_matches_projection_definition():
    for _ in range(200):
        r = rng.normal(size=(4, 3))
        phi, _ = oracle.dihedral(r)
        assert abs(phi - _projection_dihedral(r)) < 1e-10


def test_dihedral_gradient_fd_and_invariants():
    for _ in range(50):
        r = rng.normal(size=(4, 3))
        phi, g = oracle.dihedral(r)
        fd = central_fd(lambda x: oracle.dihedral(x)[0], r, 1e-6)
        assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))
        # translation and rotation invariance: zero net "force" and torque
        assert np.max(np.abs(g.sum(0))) < 1e-12 * max(1.0, np.abs(g).max())
        assert np.max(np.abs(np.cross(r, g).sum(0))) < 1e-11 * max(1.0, np.abs(g).max())
        R = rot(*rng.uniform(-3, 3, 3))
        phi2, g2 = oracle.dihedral(r @ R.T + rng.normal(size=3))
        assert abs(phi2 - phi) < 1e-10
        assert np.allclose(g2, g @ R.T, atol=1e-9)


def test_dihedral_collinear_raises():
    with pytest.raises(ValueError):
        oracle.dihedral([[0, 0, 0], [1, 0, 0], [2, 0, 0], [2, 1, 0]])


# --------------------------------------------------------------------- O2
def test_gyration_cube():
    a = 0.7
    cube = np.array(list(itertools.product([0, a], repeat=3)), dtype=np.float64) + 3.0
    rg, g = oracle.gyration(cube)
    assert abs(rg - a * math.sqrt(3) / 2) < 1e-14
    # each vertex sits at distance a*sqrt(3)/2 from the centroid
    assert np.allclose(np.linalg.norm(g, axis=1), (a * math.sqrt(3) / 2) / (8 * rg))


def test_gyration_pair_identity_fd_invariants():
    for n in (2, 3, 17, 500):
        x = rng.normal(size=(n, 3)) * 2.0
        rg, g = oracle.gyration(x)
        # Rg^2 = (1 / 2N^2) sum_ij |r_i - r_j|^2  (independent of the centroid)
        d = x[:, None, :] - x[None, :, :]
        assert abs(rg ** 2 - (d ** 2).sum() / (2 * n * n)) < 1e-12 * rg ** 2
        assert np.max(np.abs(g.sum(0))) < 1e-12
        R = rot(*rng.uniform(-3, 3, 3))
        assert abs(oracle.gyration(x @ R.T + 5.0)[0] - rg) < 1e-12 * rg
        if n <= 17:
            fd = central_fd(lambda y: oracle.gyration(y)[0], x, 1e-6)
            assert np.max(np.abs(fd - g)) < 1e-8


# --------------------------------------------------------------------- O3
def test_switch_closed_forms():
    r0 = 0.5
    s, ds = oracle.switch(r0, r0, 6, 12)
    assert s == 0.5 and abs(ds - (-1.5 / r0)) < 1e-14
    for r in [0.0, 0.01, 0.2, 0.49, 0.4999999, 0.5000001, 0.7, 1.3, 5.0]:
        s, ds = oracle.switch(r, r0, 6, 12)
        x = r / r0
        assert abs(s - 1.0 / (1.0 + x ** 6)) < 1e-15
        assert abs(ds - (-6 * x ** 5 / (1 + x ** 6) ** 2 / r0)) < 1e-13
    for n, m in [(8, 14), (6, 10), (5, 9), (1, 2)]:
        s0, d0 = oracle.switch(r0, r0, n, m)
        assert abs(s0 - n / m) < 1e-15                       # limit at r0
        assert abs(d0 - n * (n - m) / (2 * m) / r0) < 1e-13  # s'(r0) by expansion
        for r in [0.05, 0.3, 0.45, 0.6, 1.1, 2.7]:
            x = r / r0
            s, ds = oracle.switch(r, r0, n, m)
            assert abs(s - (1 - x ** n) / (1 - x ** m)) < 1e-13   # plain quotient away from r0
            fd = (oracle.switch(r + 1e-6, r0, n, m)[0] - oracle.switch(r - 1e-6, r0, n, m)[0]) / 2e-6
            assert abs(fd - ds) < 1e-7


def _cn_brute(pos, a, b, r0, n, m, rcut, L, normalize):
    """Brute force over the 27 nearest images (independent of rint)."""
    tot = 0.0
    for i in a:
        for j in b:
            if i == j:
                continue
            best = None
            shifts = [(0, 0, 0)] if L is None else itertools.product((-1, 0, 1), repeat=3)
            for s in shifts:
                d = pos[i] - pos[j] + (0 if L is None else np.array(s) * L)
                rr = np.linalg.norm(d)
                best = rr if best is None or rr < best else best
            if rcut > 0 and best >= rcut:
                continue
            x = best / r0
            tot += (1 - x ** n) / (1 - x ** m)
    return tot / len(a) if normalize else tot


def test_coordination_two_atoms_closed_form():
    pos = np.array([[0.0, 0, 0], [0.37, 0.1, -0.2]])
    cn, g = oracle.coordination(pos, [0], [1], 0.5, 6, 12)
    r = np.linalg.norm(pos[1] - pos[0])
    x = r / 0.5
    assert abs(cn - 1 / (1 + x ** 6)) < 1e-14
    dsdr = -6 * x ** 5 / (1 + x ** 6) ** 2 / 0.5
    assert np.allclose(g[0], dsdr * (pos[0] - pos[1]) / r, atol=1e-13)
    assert np.allclose(g[1], -g[0], atol=1e-15)


@pytest.mark.parametrize("box,rcut,normalize,overlap", [
    (None, 0.0, False, False), (np.array([2.0, 2.5, 3.0]), 0.0, False, False),
    (np.array([2.0, 2.0, 2.0]), 0.8, True, False), (np.array([2.0, 2.0, 2.0]), 0.0, False, True)])
def test_coordination_brute_force_fd_newton(box, rcut, normalize, overlap):
    n_atoms = 14
    pos = rng.uniform(0, 2.0, size=(n_atoms, 3))
    a = list(range(0, 6))
    b = list(range(3, 11)) if overlap else list(range(6, 12))
    cn, g = oracle.coordination(pos, a, b, 0.5, 6, 12, rcut, box, normalize)
    assert abs(cn - _cn_brute(pos, a, b, 0.5, 6, 12, rcut, box, normalize)) < 1e-12
    assert np.max(np.abs(g.sum(0))) < 1e-12          # Newton's third law
    assert np.all(g[12:] == 0.0)                      # atoms in no group
    if rcut == 0.0:
        fd = central_fd(lambda y: oracle.coordination(y, a, b, 0.5, 6, 12, rcut, box, normalize)[0], pos, 1e-6)
        assert np.max(np.abs(fd - g)) < 1e-7


def test_coordination_uniform_density_estimate():
    # raw CN per A atom ~ rho_B * 4 pi r0^3 * (pi/6) (integral of 1/(1+x^6));
    # a statistical sanity check of the sum's scale on a dense box
    g = np.random.default_rng(7)
    L = 6.0
    nb = 2000
    pos = g.uniform(0, L, size=(nb + 50, 3))
    a = list(range(nb, nb + 50))
    b = list(range(nb))
    cn, _ = oracle.coordination(pos, a, b, 0.5, 6, 12, 0.0, np.array([L, L, L]), True)
    rho = nb / L ** 3
    expect = rho * 4 * np.pi * 0.5 ** 3 * (np.pi / 6)
    # the all-pairs sum in a finite box adds a tail beyond r = L/2 that the
    # infinite-space integral also contains; allow a loose statistical margin
    assert abs(cn - expect) / expect < 0.25
