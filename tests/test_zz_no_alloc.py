"""The entry point that allocates nothing (sx_bias_eval_noalloc: partial
sums in the library's fixed device scratch) against sx_bias_eval (partial
sums in the bound workspace): the same kernels, so the same bits, on two
calls in a row, the second with a smaller input; a sample of points also
against the FP64 oracle's hill sum (V 1e-6, dV/dxi 1e-5 relative)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2301_04835_amd import Sampler, synth

from gpu_util import TWO_PI, dev, rel_inf

pytestmark = pytest.mark.gpu


def test_noalloc_bias_eval_matches_workspace_entry_point(gpu):
    sig = [0.35, 0.3]
    K0, K1 = 100000, 3000
    C0, H0 = synth.uniform_centers(K0, 2, 61), synth.uniform_heights(K0, 62)
    C1, H1 = synth.uniform_centers(K1, 2, 63), synth.uniform_heights(K1, 64)
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(0))
    s.set_walkers(np.array([0, 22, 44]), [K0 + 8, K1 + 8])
    s.metad(sig, 1.2, 300.0, 6.0, 500, 1)
    s.bind()
    s.hills_set(0, C0, H0)
    s.hills_set(1, C1, H1)
    g = np.random.default_rng(65)
    calls = [(0, g.uniform(-np.pi, np.pi, size=(70000, 2)), C0, H0),  # two batches of the 65536-point split
             (1, g.uniform(-np.pi, np.pi, size=(1000, 2)), C1, H1)]   # then a smaller call
    for w, x, C, H in calls:
        xi = dev(x)
        Vr, dVr = s.bias_eval(xi, walker=w)
        V = torch.full((x.shape[0],), float("nan"), dtype=torch.float64, device=gpu)
        dV = torch.full((x.shape[0], 2), float("nan"), dtype=torch.float64, device=gpu)
        s.bias_eval_noalloc(xi, V, dV, walker=w)
        torch.cuda.synchronize()
        assert torch.equal(V, Vr) and torch.equal(dV, dVr), w
        idx = g.choice(x.shape[0], 32, replace=False)
        Vo, dVo = oracle.hillsum_batch(x[idx], None, C.astype(np.float64), H.astype(np.float64), sig,
                                       [TWO_PI, TWO_PI], nthreads=8)
        Vh, dVh = V.cpu().numpy()[idx], dV.cpu().numpy()[idx]
        assert np.max(np.abs(Vh - Vo) / np.abs(Vo)) <= 1e-6
        assert max(rel_inf(dVh[i], dVo[i]) for i in range(32)) <= 1e-5
