"""The hand-written CV-Jacobian backward through torch.autograd, against
finite differences of the GPU forward (FP64 kernels) and the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2301_04835_amd import Sampler, synth
from paper_2301_04835_amd.autograd import cv

from gpu_util import dev, rel_inf

pytestmark = pytest.mark.gpu


def ctx_for(cvs, box=None, off=None):
    s = Sampler(0)
    s.add_cvs(cvs)
    if box is not None:
        s.set_box(box)
    if off is not None:
        s.set_walkers(off)
    s.bind()
    return s


def test_harmonic_bias_gradient_matches_fd_fp64(gpu):
    """V = k/2 sum (xi - xi0)^2 over dihedral and Rg CVs of 2 walkers
    (harmonic biasing); dV/dx from autograd vs central differences of the
    GPU forward in FP64."""
    cvs = synth.backbone_cvs(4) + [{"kind": "gyration", "idx": list(range(0, 12))}]
    W, n = 2, 22
    tmpl = synth.chain_template(n, 2)
    pos = np.concatenate([tmpl + 0.03 * np.random.default_rng(w).normal(size=tmpl.shape) for w in range(W)])
    s = ctx_for(cvs, off=np.arange(W + 1) * n)
    k = torch.tensor([100.0, 50.0, 3000.0], dtype=torch.float64, device=gpu)
    xi0 = torch.tensor([0.3, -1.0, 0.25], dtype=torch.float64, device=gpu)

    def V(p):
        return 0.5 * (k * (cv(p, s) - xi0) ** 2).sum()

    P = dev(pos).requires_grad_(True)
    e = V(P)
    e.backward()
    g = P.grad.cpu().numpy()
    fd = np.zeros_like(pos)
    h = 1e-6
    with torch.no_grad():
        for i in range(pos.shape[0]):
            for c in range(3):
                pp, pm = pos.copy(), pos.copy()
                pp[i, c] += h
                pm[i, c] -= h
                fd[i, c] = (V(dev(pp)).item() - V(dev(pm)).item()) / (2 * h)
    print("autograd vs FD:", rel_inf(g, fd))
    assert rel_inf(g, fd) <= 1e-5
    # exact chain rule with the oracle's Jacobian
    for w in range(W):
        x, J = oracle.cv_eval(pos[w * n:(w + 1) * n], cvs)
        xb = k.cpu().numpy() * (x - xi0.cpu().numpy())
        assert rel_inf(g[w * n:(w + 1) * n], np.einsum("d,dni->ni", xb, J)) <= 1e-6


def test_vjp_coordination_against_oracle(gpu):
    cvs = [{"kind": "coordination", "a": list(range(0, 300)), "b": list(range(200, 700)), "r0": 0.5, "n": 6, "m": 12,
            "rcut": 0.0, "normalize": True}]
    L = np.array([3.0, 3.0, 3.0])
    pos = np.random.default_rng(4).uniform(0, 3.0, size=(800, 3)).astype(np.float32)
    s = ctx_for(cvs, L, np.array([0, 800]))
    P = dev(pos).requires_grad_(True)
    xi = cv(P, s)
    (xi.sum() * 2.5).backward()
    x, J = oracle.cv_eval(pos.astype(np.float64), cvs, L)
    assert abs(xi.item() - x[0]) <= 1e-6 * abs(x[0])
    assert rel_inf(P.grad.cpu().numpy(), 2.5 * J[0]) <= 1e-5
