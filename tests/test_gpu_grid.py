"""GPU parity of the grid-stored metadynamics bias against the FP64 oracle
(oracle/grid.py: the exact hill sum at the nodes, multilinear read-back).

Tolerances:
  node values (FP64 sums of FP32-stored hills, exp rounding)  <= 1e-12 of
      the grid's largest |V| (|dV/dxi|); 1e-8 after deposits (a stored
      height may differ from the oracle's by one float32 rounding)
  read-back at points (same weights, FP64)                     <= 1e-12
  a step: xi <= 1e-9 rad, V <= 1e-9 relative, dV/dxi <= 1e-8 relative,
      forces <= 1e-5 relative (FP32 forces), deposited heights <= 1e-6
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.grid import BiasGrid, metad_grid_step
from paper_2301_04835_amd import Sampler, synth

from gpu_util import TWO_PI, dev, rel_inf

pytestmark = pytest.mark.gpu

KDT = oracle.KB * (6.0 - 1.0) * 300.0
PI = np.pi


def sampler(cvs, sigma, lo, hi, nbins, atom_off=None, cap=None, shared=False, stride=500, w=1.2):
    s = Sampler(0)
    s.add_cvs(cvs)
    if atom_off is not None:
        s.set_walkers(atom_off, cap, shared=shared)
    s.metad(sigma, w, 300.0, 6.0, stride, cap[0] if cap is not None else 4096)
    s.metad_grid(lo, hi, nbins)
    s.bind()
    return s


def mixed_cvs():
    """phi (periodic) and the radius of gyration of 12 atoms (not periodic)."""
    return [synth.backbone_cvs(4)[0], {"kind": "gyration", "idx": list(range(0, 12))}]


def test_nodes_and_read_back_match_oracle(gpu):
    """3,000 hills on a periodic x non-periodic grid of 64 x 40 bins: node
    values after sx_hills_set, then the read-back at random points, at
    nodes, on cell faces, on the periodic seam and outside the Rg range."""
    g = np.random.default_rng(11)
    K = 3000
    lo, hi, nb = [-PI, 0.2], [PI, 0.6], [64, 40]
    C = np.stack([g.uniform(-PI, PI, K), g.uniform(0.25, 0.55, K)], 1).astype(np.float32)
    H = g.uniform(0.5, 1.5, K).astype(np.float32)
    sigma = [0.35, 0.03]
    s = sampler(mixed_cvs(), sigma, lo, hi, nb, cap=[K + 8])
    s.hills_set(0, C, H)
    ref = BiasGrid(lo, hi, nb, [True, False])
    ref.set_hills(C.astype(np.float64), H.astype(np.float64), sigma)
    V, G = s.grid_get(0)
    assert V.size == 64 * 41
    sV, sG = np.max(np.abs(ref.V)), np.max(np.abs(ref.G))
    assert np.max(np.abs(V - ref.V.reshape(-1))) <= 1e-12 * sV
    assert np.max(np.abs(G.T - ref.G.reshape(-1, 2))) <= 1e-12 * sG
    d = ref.delta
    pts = [g.uniform([-PI, 0.2], [PI, 0.6], size=(200, 2))]
    pts.append(np.array([[lo[0] + 7 * d[0], lo[1] + 9 * d[1]], [lo[0] + 3.5 * d[0], 0.6], [PI - 0.3 * d[0], 0.41],
                         [-PI, 0.2], [PI - 1e-12, 0.33], [1.0, 0.1999], [1.0, 0.6001], [4.0, 0.3], [-9.0, 0.45]]))
    X = np.concatenate(pts)
    Vg, Gg = s.grid_eval(dev(X))
    Vg, Gg = Vg.cpu().numpy(), Gg.cpu().numpy()
    for i, x in enumerate(X):
        Vr, Gr = ref.lookup(x)
        assert abs(Vg[i] - Vr) <= 1e-12 * sV, (x, Vg[i], Vr)
        assert np.max(np.abs(Gg[i] - Gr)) <= 1e-12 * sG, (x, Gg[i], Gr)
    assert Vg[-4] == 0.0 and Vg[-3] == 0.0 and np.all(Gg[-4:-2] == 0.0)  # outside the Rg range


@pytest.mark.parametrize("stride", [5, 0])
def test_wtmd22_steps_with_grid(gpu, stride):
    """The 22-atom walker over 60 steps with a 100 x 100 grid, a deposit
    every 5 steps on top of 2,000 starting hills (or none: stride 0, where
    the step is one kernel that also moves the step counter); replayed by
    the oracle (grid rebuilt from the float32-stored list after every
    deposit)."""
    p = synth.WTMD22
    d = synth.wtmd22_inputs(n_steps=60)
    cvs = d["cvs"]
    C = d["centers"]
    H = oracle.wt_sequence(C.astype(np.float64), p["w"], KDT, p["sigma"], [TWO_PI, TWO_PI]).astype(np.float32)
    lo, hi, nb = [-PI, -PI], [PI, PI], [100, 100]
    s = sampler(cvs, list(p["sigma"]), lo, hi, nb, stride=stride, w=p["w"])
    s.hills_set(0, C, H)
    frames = dev(d["frames"])
    n = frames.shape[0]
    xi = torch.zeros((n, 2), dtype=torch.float64, device=gpu)
    V = torch.zeros(n, dtype=torch.float64, device=gpu)
    dV = torch.zeros((n, 2), dtype=torch.float64, device=gpu)
    F = torch.zeros((n, 22, 3), dtype=torch.float32, device=gpu)
    for t in range(n):
        s.step(frames[t], forces=F[t], step=t, xi_out=xi[t], V_out=V[t], dV_out=dV[t])
    s.check()
    assert s.get_step() == n
    xi, V, dV, F = (x.cpu().numpy() for x in (xi, V, dV, F))
    ref = BiasGrid(lo, hi, nb, [True, True])
    Cr, Hr = C.astype(np.float64), H.astype(np.float64)
    ref.set_hills(Cr, Hr, p["sigma"])
    worst = {"xi": 0.0, "V": 0.0, "dV": 0.0, "F": 0.0}
    for t in range(n):
        o = metad_grid_step(d["frames"][t], cvs, ref, p["w"], KDT, stride, t)
        worst["xi"] = max(worst["xi"], np.max(np.abs(xi[t] - o["xi"])))
        worst["V"] = max(worst["V"], abs(V[t] - o["V"]) / abs(o["V"]))
        worst["dV"] = max(worst["dV"], rel_inf(dV[t], o["dV"]))
        worst["F"] = max(worst["F"], rel_inf(F[t], o["F"]))
        if o["deposit"] is not None:
            Cr = np.vstack([Cr, np.float32(o["deposit"][0]).astype(np.float64)])
            Hr = np.append(Hr, float(np.float32(o["deposit"][1])))
            ref.set_hills(Cr, Hr, p["sigma"])
    print("worst errors:", worst)
    assert worst["xi"] <= 1e-9 and worst["V"] <= 1e-9 and worst["dV"] <= 1e-8 and worst["F"] <= 1e-5
    c2, h2 = s.hills_get(0)
    assert c2.shape[0] == 2000 + (n // stride if stride else 0)
    assert np.array_equal(c2[:2000], C)
    if stride:
        assert rel_inf(h2[2000:], Hr[2000:]) <= 1e-6
    Vn, _ = s.grid_get(0)
    assert np.max(np.abs(Vn - ref.V.reshape(-1))) <= 1e-8 * np.max(np.abs(ref.V))


def test_shared_list_walkers_deposit_in_order(gpu):
    """Eight walkers on one shared list and one grid, every step a deposit
    (stride 1) for 6 steps: the list holds the hills in walker order, the
    grid its exact sum, and each walker's V, dV/dxi and forces follow the
    oracle's read-back of the grid before the step."""
    W, n = 8, 22
    tmpl = synth.chain_template(n, 3)
    g = np.random.default_rng(4)
    cvs = synth.backbone_cvs(4)
    lo, hi, nb = [-PI, -PI], [PI, PI], [72, 60]
    sigma = [0.3, 0.3]
    s = sampler(cvs, sigma, lo, hi, nb, atom_off=np.arange(W + 1) * n, cap=[64], shared=True, stride=1)
    ref = BiasGrid(lo, hi, nb, [True, True])
    Cr, Hr = np.zeros((0, 2)), np.zeros(0)
    F = torch.zeros((W * n, 3), dtype=torch.float32, device=gpu)
    V = torch.zeros(W, dtype=torch.float64, device=gpu)
    dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    for t in range(6):
        pos = np.concatenate([tmpl + 0.3 * g.normal(size=tmpl.shape) for _ in range(W)])
        F.zero_()
        s.step(dev(pos), forces=F, step=t, V_out=V, dV_out=dV)
        Vg, dVg, Fg = V.cpu().numpy(), dV.cpu().numpy(), F.cpu().numpy()
        newC, newH = [], []
        for w in range(W):
            o = metad_grid_step(pos[w * n:(w + 1) * n], cvs, ref, 1.2, KDT, 1, t)
            assert abs(Vg[w] - o["V"]) <= 1e-9 * max(1.0, abs(o["V"]))
            assert rel_inf(dVg[w], o["dV"]) <= 1e-8
            assert rel_inf(Fg[w * n:(w + 1) * n], o["F"]) <= 1e-5
            newC.append(np.float32(o["deposit"][0]).astype(np.float64))
            newH.append(float(np.float32(o["deposit"][1])))
        Cr = np.vstack([Cr, newC])
        Hr = np.append(Hr, newH)
        ref.set_hills(Cr, Hr, sigma)
    s.check()
    c2, h2 = s.hills_get(0)
    assert c2.shape[0] == 6 * W
    assert rel_inf(c2, Cr) <= 1e-6 and rel_inf(h2, Hr) <= 1e-6  # float32 storage
    Vn, Gn = s.grid_get(0)
    assert np.max(np.abs(Vn - ref.V.reshape(-1))) <= 1e-8 * np.max(np.abs(ref.V))
    assert np.max(np.abs(Gn.T - ref.G.reshape(-1, 2))) <= 1e-8 * np.max(np.abs(ref.G))


def test_private_walker_outside_range_no_bias_no_deposit(gpu):
    """Two walkers with private lists on a (phi, Rg) grid whose Rg range
    excludes walker 1: walker 1 gets no bias, no force and no hill."""
    n = 22
    tmpl = synth.chain_template(n, 2)
    rg = oracle.methods.cv_eval(tmpl, mixed_cvs())[0][1]
    pos = np.concatenate([tmpl, tmpl * 3.0])  # walker 1: Rg three times larger
    s = sampler(mixed_cvs(), [0.35, 0.02], [-PI, rg - 0.1], [PI, rg + 0.1], [40, 20],
                atom_off=np.array([0, n, 2 * n]), cap=[16, 16], stride=1)
    F = torch.zeros((2 * n, 3), dtype=torch.float32, device=gpu)
    for t in range(3):
        s.step(dev(pos), forces=F, step=t)
    s.check()
    assert s.hill_counts().tolist() == [3, 0]
    Fh = F.cpu().numpy()
    assert np.all(Fh[n:] == 0.0) and np.max(np.abs(Fh[:n])) > 0.0


def test_grid_arguments(gpu):
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(4))
    with pytest.raises(Exception):
        s.metad_grid([-PI, -PI], [PI, 3.0], [10, 10])  # a periodic CV needs one period
    with pytest.raises(Exception):
        s.metad_grid([-PI, -PI], [PI, PI], [1, 10])
    s.metad_grid([-PI, -PI], [PI, PI], [10, 10])
    s.abf([-PI, -PI], [PI, PI], [10, 10])
    with pytest.raises(Exception):
        s.bind()  # a grid bias needs metadynamics


def test_graph_replay_matches_eager_steps(gpu):
    """A captured 3-step graph of the grid path (shared list of 4 walkers,
    a deposit every 2 steps, device step counter), replayed four times,
    against the same steps run eagerly: forces, V, the hill list and the
    grid agree bitwise."""
    W, n = 4, 22
    tmpl = synth.chain_template(n, 5)
    pos = np.concatenate([tmpl + 0.2 * np.random.default_rng(w).normal(size=tmpl.shape) for w in range(W)])
    C = synth.uniform_centers(300, 2, 6)
    H = synth.uniform_heights(300, 7)
    mk = lambda: sampler(synth.backbone_cvs(4), [0.35, 0.35], [-PI, -PI], [PI, PI], [48, 48],
                         atom_off=np.arange(W + 1) * n, cap=[400], shared=True, stride=2)
    a, b = mk(), mk()
    a.hills_set(0, C, H)
    b.hills_set(0, C, H)
    P = dev(pos)
    Fa = torch.zeros((W * n, 3), dtype=torch.float32, device=gpu)
    Fb = torch.zeros_like(Fa)
    Va = torch.zeros(W, dtype=torch.float64, device=gpu)
    Vb = torch.zeros_like(Va)
    a.graph_capture(3, P, forces=Fa, V_out=Va)
    for rep in range(4):
        a.graph_launch()
        torch.cuda.synchronize()
        for _ in range(3):
            b.step(P, forces=Fb, V_out=Vb)
        torch.cuda.synchronize()
        assert torch.equal(Fa, Fb) and torch.equal(Va, Vb), rep
    assert a.get_step() == 12 and b.get_step() == 12
    ca, ha = a.hills_get(0)
    cb, hb = b.hills_get(0)
    assert ca.shape[0] == 300 + 6 * W and np.array_equal(ca, cb) and np.array_equal(ha, hb)
    Ga, Gb = a.grid_get(0), b.grid_get(0)
    assert np.array_equal(Ga[0], Gb[0]) and np.array_equal(Ga[1], Gb[1])


@pytest.mark.parametrize("D", [1, 3])
def test_nodes_and_read_back_one_and_three_cvs(gpu, D):
    """D = 1 (phi) and D = 3 (phi, psi, Rg of 12 atoms): node values after
    sx_hills_set and the read-back at random points, against the oracle."""
    g = np.random.default_rng(30 + D)
    if D == 1:
        cvs, per = synth.backbone_cvs(4)[:1], [True]
        lo, hi, nb, sigma = [-PI], [PI], [80], [0.3]
        C = g.uniform(-PI, PI, size=(500, 1))
    else:
        cvs = synth.backbone_cvs(4) + [{"kind": "gyration", "idx": list(range(0, 12))}]
        per = [True, True, False]
        lo, hi, nb, sigma = [-PI, -PI, 0.2], [PI, PI, 0.6], [24, 20, 10], [0.35, 0.35, 0.04]
        C = np.concatenate([g.uniform(-PI, PI, size=(800, 2)), g.uniform(0.25, 0.55, size=(800, 1))], 1)
    C = C.astype(np.float32)
    H = g.uniform(0.5, 1.5, len(C)).astype(np.float32)
    s = sampler(cvs, sigma, lo, hi, nb, cap=[len(C) + 8])
    s.hills_set(0, C, H)
    ref = BiasGrid(lo, hi, nb, per)
    ref.set_hills(C.astype(np.float64), H.astype(np.float64), sigma)
    V, G = s.grid_get(0)
    sV, sG = np.max(np.abs(ref.V)), np.max(np.abs(ref.G))
    assert np.max(np.abs(V - ref.V.reshape(-1))) <= 1e-12 * sV
    assert np.max(np.abs(G.T - ref.G.reshape(-1, D))) <= 1e-12 * sG
    X = g.uniform(lo, hi, size=(300, D))
    Vg, Gg = s.grid_eval(dev(X))
    Vg, Gg = Vg.cpu().numpy(), Gg.cpu().numpy()
    for i, x in enumerate(X):
        Vr, Gr = ref.lookup(x)
        assert abs(Vg[i] - Vr) <= 1e-12 * sV
        assert np.max(np.abs(Gg[i] - Gr)) <= 1e-12 * sG
