"""GPU parity of harmonic biasing and the umbrella-integration windows
against the FP64 oracle (oracle/umbrella.py).

Tolerances: V and dV/dxi <= 1e-9 relative (FP64 CVs and spring on both
sides), forces <= 1e-5 relative (FP32 forces), window means and
covariances <= 1e-10 of their scale (FP64 sums in step order), mean forces
and A <= 1e-9; graph replay bitwise equal to eager steps.
"""
import numpy as np
import pytest
import torch

from oracle import methods
from oracle.umbrella import Window, harmonic, integrate
from paper_2301_04835_amd import Sampler, synth

from gpu_util import dev, rel_inf

pytestmark = pytest.mark.gpu

PI = np.pi


def windows(W, cvs, k, centers, n=22):
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_walkers(np.arange(W + 1) * n)
    s.harmonic(k, centers)
    s.bind()
    return s


@pytest.mark.parametrize("mixed", [False, True])
def test_steps_windows_and_integration_match_oracle(gpu, mixed):
    """16 windows along a path in (phi, psi) -- the first ones straddling the
    periodic seam -- or in (phi, Rg); 25 steps of jittered chains; per step
    V, dV/dxi and forces, then the window moments and the integrated
    profile."""
    W, n, steps = 16, 22, 25
    cvs = synth.backbone_cvs(4) if not mixed else [synth.backbone_cvs(4)[0],
                                                   {"kind": "gyration", "idx": list(range(0, 12))}]
    per = [True, not mixed]
    tmpl = [synth.chain_template(n, 10 + w) for w in range(W)]
    xi_t = np.array([methods.cv_eval(t, cvs)[0] for t in tmpl])
    # centres: the template's CVs shifted along a path; windows 0-2 sit
    # across the seam from their walkers
    shift = np.stack([np.linspace(-0.3, 0.3, W), np.linspace(0.2, -0.2, W) * (0.1 if mixed else 1.0)], 1)
    centers = xi_t + shift
    centers[:3, 0] = np.where(xi_t[:3, 0] > 0, xi_t[:3, 0] - 2 * PI + 0.1, xi_t[:3, 0] + 2 * PI - 0.1)
    k = np.array([120.0, 80.0 if not mixed else 2000.0])
    s = windows(W, cvs, k, centers)
    g = np.random.default_rng(1)
    wins = [Window(2) for _ in range(W)]
    F = torch.zeros((W * n, 3), dtype=torch.float32, device=gpu)
    V = torch.zeros(W, dtype=torch.float64, device=gpu)
    dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    for t in range(steps):
        pos = np.concatenate([tm + 0.02 * g.normal(size=tm.shape) for tm in tmpl])
        F.zero_()
        s.step(dev(pos), forces=F, step=t, V_out=V, dV_out=dV)
        Vg, dVg, Fg = V.cpu().numpy(), dV.cpu().numpy(), F.cpu().numpy()
        for w in range(W):
            xi, J = methods.cv_eval(pos[w * n:(w + 1) * n], cvs)
            Vr, dVr, Dv = harmonic(xi, centers[w], k, per)
            assert abs(Vg[w] - Vr) <= 1e-9 * abs(Vr)
            assert rel_inf(dVg[w], dVr) <= 1e-9
            assert rel_inf(Fg[w * n:(w + 1) * n], methods.chain_rule(-dVr, J)) <= 1e-5
            wins[w].add(Dv)
    s.check()
    assert s.get_step() == steps
    nn, m, C = s.umbrella_stats()
    assert np.all(nn == steps)
    for w in range(W):
        mr, Cr = wins[w].mean_cov(centers[w])
        assert np.max(np.abs(m[w] - mr)) <= 1e-10 * max(1.0, np.max(np.abs(mr)))
        assert np.max(np.abs(C[w] - Cr)) <= 1e-10 * max(1e-6, np.max(np.abs(Cr)))
    gf, A = s.umbrella_integrate()
    gr, Ar = integrate([wins[w].mean_cov(centers[w])[0] for w in range(W)], centers, k, per)
    assert np.max(np.abs(gf - gr)) <= 1e-9 * np.max(np.abs(gr))
    assert np.max(np.abs(A - Ar)) <= 1e-9 * max(1.0, np.max(np.abs(Ar)))
    s.umbrella_reset()
    assert np.all(s.umbrella_stats()[0] == 0)


def test_graph_replay_matches_eager_steps(gpu):
    W, n = 6, 22
    cvs = synth.backbone_cvs(4)
    pos = np.concatenate([synth.chain_template(n, 40 + w) for w in range(W)])
    centers = np.random.default_rng(2).uniform(-PI, PI, size=(W, 2))
    a = windows(W, cvs, [50.0, 70.0], centers)
    b = windows(W, cvs, [50.0, 70.0], centers)
    P = dev(pos)
    Fa = torch.zeros((W * n, 3), dtype=torch.float32, device=gpu)
    Fb = torch.zeros_like(Fa)
    a.graph_capture(4, P, forces=Fa)
    for rep in range(3):
        a.graph_launch()
        for _ in range(4):
            b.step(P, forces=Fb)
        torch.cuda.synchronize()
        assert torch.equal(Fa, Fb), rep
    assert a.get_step() == 12 and b.get_step() == 12
    sa, sb = a.umbrella_stats(), b.umbrella_stats()
    assert all(np.array_equal(x, y) for x, y in zip(sa, sb)) and np.all(sa[0] == 12)


def test_harmonic_arguments(gpu):
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(4))
    with pytest.raises(Exception):
        s.harmonic([0.0, 1.0], [[0.0, 0.0]])
    s.set_walkers(np.array([0, 22, 44]))
    s.harmonic([1.0, 1.0], [[0.0, 0.0]])  # one centre for two walkers
    with pytest.raises(Exception):
        s.bind()
    t = Sampler(0)
    t.add_cvs(synth.backbone_cvs(4))
    t.harmonic([1.0, 1.0], [[0.0, 0.0]])
    with pytest.raises(Exception):
        t.metad([0.3, 0.3], 1.0)
