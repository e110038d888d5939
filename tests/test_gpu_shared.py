"""GPU parity of the shared-hill-list sum (walkers sharing one bias, and the
bias evaluated at arbitrary query points) against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2301_04835_amd import Sampler, synth
from paper_2301_04835_amd.api import SxError

from gpu_util import TWO_PI, dev, rel_inf

pytestmark = pytest.mark.gpu

KDT = oracle.KB * 5 * 300.0


def shared_ctx(cvs, sigma, W, n_atoms, cap, stride=500, bias_factor=6.0):
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_walkers(np.arange(W + 1) * n_atoms, [cap], shared=True)
    s.metad(sigma, 1.2, 300.0, bias_factor, stride, cap)
    s.bind()
    return s


@pytest.mark.parametrize("K", [5000, 20000])
def test_shared_list_walkers_step_and_deposit(gpu, K):
    """K = 5,000: few chunk records per walker (one lane per walker sums
    them); K = 20,000: more than 32 (one wavefront per walker, the force
    table in the kernel arguments); both with the step-0 deposit and the
    full list's capacity report."""
    W, n = 24, 12
    cvs = synth.backbone_cvs(1)
    tmpl = synth.chain_template(n, 4)
    pos = np.concatenate([tmpl + np.random.default_rng(w).normal(0, 0.2, tmpl.shape) for w in range(W)])
    C = synth.uniform_centers(K, 2, 21)
    H = synth.uniform_heights(K, 22)
    s = shared_ctx(cvs, [0.35, 0.3], W, n, K + W)
    s.hills_set(-1, C, H)
    P = dev(pos.astype(np.float32))
    F = torch.zeros_like(P)
    xi = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    V = torch.zeros(W, dtype=torch.float64, device=gpu)
    dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    s.step(P, forces=F, step=0, xi_out=xi, V_out=V, dV_out=dV)
    s.check()
    xr, Js = np.zeros((W, 2)), []
    for w in range(W):
        xr[w], J = oracle.cv_eval(pos[w * n:(w + 1) * n].astype(np.float32).astype(np.float64), cvs)
        Js.append(J)
    Vr, dVr = oracle.hillsum_batch(xr, None, C.astype(np.float64), H.astype(np.float64), [0.35, 0.3], [TWO_PI] * 2,
                                   nthreads=8)
    assert np.max(np.abs(xi.cpu().numpy() - xr)) <= 1e-9
    assert np.max(np.abs(V.cpu().numpy() - Vr) / Vr) <= 1e-6
    Fh = F.cpu().numpy()
    for w in range(W):
        assert rel_inf(dV.cpu().numpy()[w], dVr[w]) <= 1e-5
        assert rel_inf(Fh[w * n:(w + 1) * n], oracle.chain_rule(-dVr[w], Js[w])) <= 1e-5
    # step 0 deposited W hills in walker order with the WT height of each walker
    c2, h2 = s.hills_get(-1)
    assert c2.shape[0] == K + W
    assert np.array_equal(c2[K:], xr.astype(np.float32))
    assert rel_inf(h2[K:], 1.2 * np.exp(-Vr / KDT)) <= 1e-6
    # the list is now full: the next deposit appends nothing and reports it
    s.step(P, forces=F, step=500)
    with pytest.raises(SxError) as ei:
        s.check()
    assert ei.value.status == 3
    assert s.hills_get(-1)[0].shape[0] == K + W


@pytest.mark.parametrize("shared", [False, True])
def test_bias_eval_many_points_2d(gpu, shared):
    K, n = 3000, 70000  # two batches of query points
    C = synth.uniform_centers(K, 2, 31)
    H = synth.uniform_heights(K, 32)
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(0))
    if shared:
        s.set_walkers([0, 8, 16], [K], shared=True)
    s.metad([0.3, 0.3], 1.0, 300.0, None, 0, K)
    s.bind()
    s.hills_set(0, C, H)
    q = np.random.default_rng(5).uniform(-np.pi, np.pi, size=(n, 2))
    V, dV = s.bias_eval(dev(q))
    idx = np.random.default_rng(6).choice(n, 4000, replace=False)
    Vr, dVr = oracle.hillsum_batch(q[idx], None, C.astype(np.float64), H.astype(np.float64), [0.3, 0.3],
                                   [TWO_PI] * 2, nthreads=8)
    Vh, dVh = V.cpu().numpy()[idx], dV.cpu().numpy()[idx]
    assert np.max(np.abs(Vh - Vr) / np.abs(Vr)) <= 1e-6
    scale = np.max(np.abs(dVr), axis=1)
    assert np.max(np.max(np.abs(dVh - dVr), axis=1) / scale) <= 1e-5


def test_bias_eval_3d_nonperiodic_and_empty(gpu):
    """Three non-periodic CVs (coordination-like values), sigma 0.2."""
    cvs = [{"kind": "gyration", "idx": [0, 1, 2]}, {"kind": "gyration", "idx": [3, 4, 5]},
           {"kind": "gyration", "idx": [6, 7, 8]}]
    K = 4000
    g = np.random.default_rng(9)
    C = (9.0 + 0.3 * g.normal(size=(K, 3))).astype(np.float32)
    H = synth.uniform_heights(K, 10)
    s = Sampler(0)
    s.add_cvs(cvs)
    s.metad([0.2, 0.2, 0.2], 1.0, 300.0, None, 0, K + 1)
    s.bind()
    q = 9.0 + 0.4 * g.normal(size=(3000, 3))
    V0, _ = s.bias_eval(dev(q))
    assert torch.all(V0 == 0)  # no hills yet
    s.hills_set(0, C, H)
    V, dV = s.bias_eval(dev(q))
    Vr, dVr = oracle.hillsum_batch(q, None, C.astype(np.float64), H.astype(np.float64), [0.2] * 3, [0.0] * 3,
                                   nthreads=8)
    m = Vr > 1e-3 * Vr.max()
    assert np.max(np.abs(V.cpu().numpy()[m] - Vr[m]) / Vr[m]) <= 1e-6
    scale = np.max(np.abs(dVr), axis=1)
    mm = scale > 1e-3 * scale.max()
    assert np.max((np.max(np.abs(dV.cpu().numpy() - dVr), axis=1) / scale)[mm]) <= 1e-5
