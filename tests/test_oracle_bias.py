"""Pins of the FP64 oracle's hill sum, well-tempered deposition, chain rule
and ABF bookkeeping (no GPU)."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2301_04835_amd import synth

rng = np.random.default_rng(2024)
TWO_PI = 2 * np.pi


# --------------------------------------------------------------------- O4
def test_single_hill_closed_form():
    xi = np.array([0.3, -1.2])
    c = np.array([[0.1, -0.9]])
    h = np.array([1.7])
    sig = np.array([0.35, 0.5])
    V, dV = oracle.hillsum(xi, c, h, sig, [TWO_PI, TWO_PI])
    d = xi - c[0]
    e = 1.7 * math.exp(-(d[0] ** 2 / (2 * 0.35 ** 2) + d[1] ** 2 / (2 * 0.5 ** 2)))
    assert abs(V - e) < 1e-15
    assert np.allclose(dV, [-e * d[0] / 0.35 ** 2, -e * d[1] / 0.5 ** 2], atol=1e-15)


def test_hill_wrap_across_boundary():
    # xi near +pi, hill near -pi: the minimum image distance is small
    xi = np.array([np.pi - 0.05])
    V, dV = oracle.hillsum(xi, [[-np.pi + 0.05]], [1.0], [0.3], [TWO_PI])
    assert abs(V - math.exp(-0.1 ** 2 / (2 * 0.09))) < 1e-14
    assert dV[0] > 0  # the hill lies "ahead" of xi across the boundary
    # a non-periodic CV sees the full distance
    V2, _ = oracle.hillsum(xi, [[-np.pi + 0.05]], [1.0], [0.3], [0.0])
    assert V2 < 1e-40


def test_hillsum_fd_periodicity_images():
    K = 300
    c = rng.uniform(-np.pi, np.pi, size=(K, 2))
    h = rng.uniform(0.5, 1.5, size=K)
    sig = np.array([0.35, 0.3])
    per = np.array([TWO_PI, TWO_PI])
    for _ in range(20):
        xi = rng.uniform(-np.pi, np.pi, size=2)
        V, dV = oracle.hillsum(xi, c, h, sig, per)
        fd = np.array([(oracle.hillsum(xi + e * 1e-5, c, h, sig, per)[0] -
                        oracle.hillsum(xi - e * 1e-5, c, h, sig, per)[0]) / 2e-5 for e in np.eye(2)])
        assert np.max(np.abs(fd - dV)) < 1e-7 * max(1, np.abs(dV).max())
        for e in np.eye(2):
            assert abs(oracle.hillsum(xi + TWO_PI * e, c, h, sig, per)[0] - V) < 1e-12 * V
        # 3^D image sum (no wrap, explicit copies) equals the minimum image
        Vimg = 0.0
        for s in itertools.product((-1, 0, 1), repeat=2):
            Vimg += oracle.hillsum(xi, c + TWO_PI * np.array(s), h, sig, [0.0, 0.0])[0]
        assert abs(Vimg - V) < 1e-13 * V


def test_symmetric_hills_zero_gradient_3d_nonperiodic():
    x0 = np.array([0.4, -0.2, 1.1])
    a = 0.23
    c = [x0 + s * a * e for e in np.eye(3) for s in (-1, 1)]
    V, dV = oracle.hillsum(x0, c, np.ones(6), [0.2, 0.3, 0.25], [0, 0, 0])
    assert np.max(np.abs(dV)) < 1e-14
    assert V > 0


def test_hillsum_batch_matches_loop_private_and_shared():
    W, D = 5, 2
    counts = np.array([3, 0, 7, 1, 4])
    off = np.concatenate([[0], np.cumsum(counts)])
    c = rng.uniform(-3, 3, size=(off[-1], D))
    h = rng.uniform(0.5, 1.5, off[-1])
    xi = rng.uniform(-3, 3, size=(W, D))
    sig, per = [0.35, 0.35], [TWO_PI, 0.0]
    V, dV = oracle.hillsum_batch(xi, off, c, h, sig, per, nthreads=3)
    for w in range(W):
        v1, d1 = oracle.hillsum(xi[w], c[off[w]:off[w + 1]], h[off[w]:off[w + 1]], sig, per)
        assert V[w] == v1 and np.array_equal(dV[w], d1)
    Vs, _ = oracle.hillsum_batch(xi, None, c, h, sig, per)
    for w in range(W):
        assert Vs[w] == oracle.hillsum(xi[w], c, h, sig, per)[0]


# --------------------------------------------------------------------- O5
def test_wt_repeated_point_recurrence():
    # all hills at one point: V_k(s) = sum_{j<k} h_j, a scalar recurrence
    w, kdT = 1.2, oracle.KB * 5 * 300.0
    c = np.zeros((50, 2)) + 0.3
    h = oracle.wt_sequence(c, w, kdT, [0.35, 0.35], [TWO_PI, TWO_PI], round_f32=False)
    acc = 0.0
    for k in range(50):
        hk = w * math.exp(-acc / kdT)
        assert abs(h[k] - hk) < 1e-13
        acc += hk
    # plain metadynamics: constant height
    h2 = oracle.wt_sequence(c, w, 0.0, [0.35, 0.35], [TWO_PI, TWO_PI])
    assert np.all(h2 == np.float32(w))
    assert oracle.wt_height(w, 123.0, math.inf) == w


def test_wt_sequence_round_f32_and_growth_law():
    w, kdT = 1.2, oracle.KB * 5 * 300.0
    c = rng.uniform(-np.pi, np.pi, size=(400, 2))
    h = oracle.wt_sequence(c, w, kdT, [0.35, 0.35], [TWO_PI] * 2, round_f32=True)
    assert np.all(h.astype(np.float32).astype(np.float64) == h)
    assert np.all(h <= np.float32(w)) and np.all(h > 0)
    # continuum well-tempered growth for uniform deposits on the torus:
    # dV/dk = a w exp(-V/c) with a = 2 pi s1 s2 / (2 pi)^2  =>  V = c ln(1 + a w k / c)
    a = 2 * np.pi * 0.35 * 0.35 / TWO_PI ** 2
    Vmean = np.mean([oracle.hillsum(x, c, h, [0.35] * 2, [TWO_PI] * 2)[0]
                     for x in rng.uniform(-np.pi, np.pi, size=(400, 2))])
    Vlaw = kdT * math.log(1 + a * w * 400 / kdT)
    assert abs(Vmean - Vlaw) / Vlaw < 0.1


def test_paper_parameter_table_fixture():
    """The metadynamics settings of the appendix table drive the same law;
    butane's WTMD gives dT = 5000 K directly."""
    import json
    import os
    p = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))
    assert p["adp"]["metadynamics"] == {"sigma_rad": 0.35, "height_kJmol": 1.2, "stride": 500}
    b = p["butane"]["wtmd"]
    kdT = oracle.KB * b["delta_T_K"]
    assert abs(kdT - 41.57231309) < 1e-8
    h = oracle.wt_sequence(np.zeros((3, 1)), b["height_kJmol"], kdT, [b["sigma_rad"]], [TWO_PI], False)
    assert abs(h[1] - b["height_kJmol"] * math.exp(-b["height_kJmol"] / kdT)) < 1e-16
    assert p["adp"]["abf_threshold_N"] == 500
    assert p["adp"]["grid_points_per_cv"] == 50 and p["butane"]["grid_points_per_cv"] == 64


# --------------------------------------------------------------------- O6
def test_metad_step_force_is_minus_gradient():
    d = synth.wtmd22_inputs(n_steps=2)
    x = d["frames"][0]
    cvs = d["cvs"]
    c = d["centers"][:200].astype(np.float64)
    h = rng.uniform(0.5, 1.5, 200)
    sig = [0.35, 0.35]
    out = oracle.metad_step(x, cvs, c, h, sig, 1.2, 0.0, 500, 3)
    assert out["deposit"] is None

    def energy(y):
        xi, _ = oracle.cv_eval(y, cvs)
        return oracle.hillsum(xi, c, h, sig, [TWO_PI, TWO_PI])[0]

    F = out["F"]
    touched = sorted(set(cvs[0]["idx"]) | set(cvs[1]["idx"]))
    for i in touched:
        for k in range(3):
            yp, ym = x.copy(), x.copy()
            yp[i, k] += 1e-6
            ym[i, k] -= 1e-6
            assert abs(-(energy(yp) - energy(ym)) / 2e-6 - F[i, k]) < 1e-6 * max(1, np.abs(F).max())
    assert np.all(F[[i for i in range(22) if i not in touched]] == 0)
    assert np.max(np.abs(F.sum(0))) < 1e-10 * np.abs(F).max()
    assert np.max(np.abs(np.cross(x, F).sum(0))) < 1e-10 * np.abs(F).max()
    dep = oracle.metad_step(x, cvs, c, h, sig, 1.2, oracle.KB * 1500, 500, 1000)["deposit"]
    assert np.array_equal(dep[0], out["xi"])
    assert abs(dep[1] - 1.2 * math.exp(-out["V"] / (oracle.KB * 1500))) < 1e-15


# --------------------------------------------------------------------- O7
def test_abf_theta_linear_cv():
    # xi = a . x for a linear CV: J = a, theta = -(a.F)/|a|^2
    a = rng.normal(size=(1, 4, 3))
    F = rng.normal(size=(4, 3))
    th = oracle.abf_theta(a, F)
    assert abs(th[0] - (-(a[0] * F).sum() / (a[0] ** 2).sum())) < 1e-13
    # two orthogonal linear CVs decouple
    b = np.zeros((2, 4, 3))
    b[0, 0, 0] = 2.0
    b[1, 1, 2] = -3.0
    th2 = oracle.abf_theta(b, F)
    assert np.allclose(th2, [-F[0, 0] / 2.0, F[1, 2] / 3.0], atol=1e-15)
    # a force purely along the gradient of xi is recovered exactly
    c = rng.normal(size=(2, 5, 3))
    t0 = np.array([0.7, -1.3])
    Fpar = -np.einsum("d,dni->ni", t0, c)
    assert np.allclose(oracle.abf_theta(c, Fpar), t0, atol=1e-12)


def test_abf_bins():
    # exactly representable edges so that each decision below is unambiguous
    lo, hi, nb = [-2.0, 0.0], [2.0, 10.0], [8, 20]
    per = [True, False]
    assert oracle.abf_bin([-2.0, 0.0], lo, hi, nb, per) == 0
    assert oracle.abf_bin([2.0, 0.0], lo, hi, nb, per) == 0            # wraps
    assert oracle.abf_bin([0.0, 9.75], lo, hi, nb, per) == 4 * 20 + 19
    assert oracle.abf_bin([0.0, 10.0], lo, hi, nb, per) == -1          # half-open
    assert oracle.abf_bin([0.0, -0.25], lo, hi, nb, per) == -1
    assert oracle.abf_bin([-2.25, 5.0], lo, hi, nb, per) == 7 * 20 + 10
    assert oracle.abf_bin([2.25, 0.5], lo, hi, nb, per) == 0 * 20 + 1


def test_abf_constant_sample_replay_and_counts():
    g = oracle.AbfGrid([0.0], [1.0], [4], [False], n_threshold=5)
    J = np.zeros((1, 2, 3))
    J[0, 0, 0] = 1.0
    F = np.zeros((2, 3))
    F[0, 0] = -2.0  # theta = 2
    bs = []
    for M in range(8):
        b, Fb, k, th = oracle.abf_step(g, [0.3], J, F)
        assert k == 1 and th[0] == 2.0
        assert b[0] == M * 2.0 / max(M, 5)
        assert Fb[0, 0] == b[0] and np.all(Fb[1] == 0)
        bs.append(b[0])
    b, Fb, k, _ = oracle.abf_step(g, [1.5], J, F)  # out of range: dropped
    assert k == -1 and b[0] == 0.0 and np.all(Fb == 0)
    assert g.N.sum() == 8 and g.N[1] == 8 and g.Fsum[1, 0] == 16.0
