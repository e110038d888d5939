"""GPU-side free-energy analysis against the oracle (oracle/analysis.py).

  metadynamics FES at analysis-grid nodes (the evaluation kernel's bar:
      FP32 Gaussians, FP64 sums, V <= 1e-6 relative; F and the oracle's
      are each shifted by their own minimum)   <= 2e-6 of max |F|
  ABF FES from the library's grid (host CG vs dense least squares on the
      same counts and sums)                                   <= 1e-8 of its range
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.analysis import abf_fes, metad_fes
from paper_2301_04835_amd import Sampler, synth

from gpu_util import dev

pytestmark = pytest.mark.gpu

PI = np.pi
TWO_PI = 2.0 * PI


def test_metad_fes_matches_oracle(gpu):
    """Well-tempered and plain factors on a (phi, Rg) bias of 600 hills."""
    cvs = [synth.backbone_cvs(4)[0], {"kind": "gyration", "idx": list(range(0, 12))}]
    g = np.random.default_rng(3)
    C = np.stack([g.uniform(-PI, PI, 600), g.uniform(0.3, 0.5, 600)], 1).astype(np.float32)
    H = g.uniform(0.5, 1.5, 600).astype(np.float32)
    sigma = [0.35, 0.02]
    lo, hi, nb = [-PI, 0.25], [PI, 0.55], [36, 30]
    for gamma in (6.0, None):
        s = Sampler(0)
        s.add_cvs(cvs)
        s.metad(sigma, 1.2, 300.0, gamma, 0, 700)
        s.bind()
        s.hills_set(0, C, H)
        F = s.metad_fes(lo, hi, nb, temperature=300.0)
        kdT = oracle.KB * 300.0 * (gamma - 1.0) if gamma else 0.0
        Fr = metad_fes(C.astype(np.float64), H.astype(np.float64), sigma, [TWO_PI, 0.0], lo, hi, nb, [True, False],
                       300.0, kdT)
        assert F.shape == Fr.shape == (36, 31)
        assert np.max(np.abs(F - Fr)) <= 2e-6 * np.max(np.abs(Fr))


def test_abf_fes_matches_oracle(gpu):
    """ABF on (phi, psi) of 8 walkers of jittered chains with random system
    forces, 400 steps on a 12 x 10 grid; the library's integration of each
    walker's grid against the oracle's on the same counts and sums."""
    W, n = 8, 22
    cvs = synth.backbone_cvs(4)
    nb = [12, 10]
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_walkers(np.arange(W + 1) * n)
    s.abf([-PI, -PI], [PI, PI], nb, 5)
    s.bind()
    g = np.random.default_rng(5)
    tmpl = [synth.chain_template(n, 60 + w) for w in range(W)]
    F = torch.zeros((W * n, 3), dtype=torch.float32, device=gpu)
    for t in range(400):
        pos = np.concatenate([tm + 0.25 * g.normal(size=tm.shape) for tm in tmpl]).astype(np.float32)
        fs = (50.0 * g.normal(size=pos.shape)).astype(np.float32)
        s.step(dev(pos), forces=F, step=t, sys_forces=dev(fs))
    s.check()
    delta = [TWO_PI / nb[0], TWO_PI / nb[1]]
    for w in range(W):
        N, Fsum = s.abf_grid(w)
        A = s.abf_fes(w)
        Ar = abf_fes(N.reshape(-1), Fsum.reshape(-1, 2), nb, delta, [True, True])
        vis = N.reshape(nb) > 0
        assert vis.sum() > 0.8 * vis.size  # most bins visited
        assert np.array_equal(np.isnan(A), ~vis)
        scale = max(1.0, np.nanmax(Ar))
        assert np.nanmax(np.abs(A - Ar)) <= 1e-8 * scale
