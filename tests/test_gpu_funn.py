"""FUNN on the GPU: a network fitted to ABF mean forces, whose gradient then
biases the ABF run (oracle: oracle/mlp.py on the same bf16 weights, and the
oracle's Jacobians for the forces).

  the fitted network's gradient at the bin centres vs the oracle network
      (the kernel's arithmetic)                                 <= 2e-5
  the fit itself: rms |grad A_net - g| over the visited bins    <= 0.1 rms |g|
  a FUNN step: b = the network gradient at xi                  bitwise equal
      to sx_surrogate_eval's; forces the chain rule of b        <= 1e-5
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from paper_2301_04835_amd import Sampler, synth

from gpu_util import dev, rel_inf

pytestmark = pytest.mark.gpu

PI = np.pi


def grad_A(x):
    """A(phi, psi) = 3 cos(phi - 1) + 2 cos(psi + 0.5) + cos(phi + psi)."""
    return np.array([-3 * np.sin(x[0] - 1) - np.sin(x[0] + x[1]), -2 * np.sin(x[1] + 0.5) - np.sin(x[0] + x[1])])


def test_funn_fit_and_bias(gpu):
    W, n, H = 4, 22, 64
    cvs = synth.backbone_cvs(4)
    nb = [16, 16]
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_walkers(np.arange(W + 1) * n)
    s.abf([-PI, -PI], [PI, PI], nb, 1)
    s.surrogate(H, max_samples=1024, max_batch=1024, cert_n=8, tol_force=0.1)
    s.bind()
    # fill the grid with the mean force of A: system forces -J^T grad A(xi)
    g = np.random.default_rng(9)
    tmpl = [synth.chain_template(n, 90 + w) for w in range(W)]
    F = torch.zeros((W * n, 3), dtype=torch.float32, device=gpu)
    for t in range(700):
        pos = np.concatenate([tm + 0.3 * g.normal(size=tm.shape) for tm in tmpl])
        fs = np.zeros_like(pos)
        for w in range(W):
            xi, J = oracle.cv_eval(pos[w * n:(w + 1) * n], cvs)
            fs[w * n:(w + 1) * n] = -np.einsum("d,dni->ni", grad_A(xi), J)
        s.step(dev(pos.astype(np.float32)), forces=F, step=t, sys_forces=dev(fs.astype(np.float32)))
    s.check()
    N, Fsum = s.abf_grid(0)
    vis = N > 0
    assert vis.sum() > 150
    P0 = mlp.init_params(H, 4, 3)
    s.surrogate_params(np.concatenate([np.ravel(P0[k]) for k in mlp.PARAM_ORDER]).astype(np.float32))
    s.surrogate_output(3.0, 0.0)
    used, loss = s.funn_fit(walker=0, batch=1024, steps=4000, lr=3e-3, lr_final=1e-5)
    assert used == vis.sum()
    # network gradient at the visited bin centres
    ii, jj = np.nonzero(vis.reshape(nb))
    d = 2 * PI / 16
    X = np.stack([-PI + (ii + 0.5) * d, -PI + (jj + 0.5) * d], 1)
    _, dVn = s.surrogate_eval(dev(X))
    dVn = dVn.cpu().numpy()
    Pf = s.surrogate_params()
    shapes = [("W1", (H, 4)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
    Pd, o = {}, 0
    for k, sh in shapes:
        m = int(np.prod(sh))
        Pd[k] = mlp.round_bf16(np.asarray(Pf[o:o + m], dtype=np.float64).reshape(sh))
        o += m
    _, dy, _ = mlp.forward(Pd, X, [True, True], act_round=mlp.round_bf16x2)
    assert np.max(np.abs(dVn - 3.0 * dy)) <= 2e-5 * np.max(np.abs(3.0 * dy))
    gbin = (Fsum[vis] / N[vis][:, None])
    rms = np.sqrt(np.mean(np.sum((dVn - gbin) ** 2, 1)) / np.mean(np.sum(gbin ** 2, 1)))
    print("FUNN fit: visited", used, "loss", loss, "relative rms gradient error", rms)
    assert rms <= 0.1
    # a FUNN step: the bias is the network's gradient at xi
    s.funn_enable(True)
    Nbefore = N.sum()
    pos = np.concatenate([tm + 0.3 * g.normal(size=tm.shape) for tm in tmpl]).astype(np.float32)
    xi_o = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    F.zero_()
    s.step(dev(pos), forces=F, step=700, xi_out=xi_o, dV_out=dV, sys_forces=dev(np.zeros_like(pos)))
    s.check()
    _, dVe = s.surrogate_eval(xi_o)
    assert torch.equal(-dV, dVe)
    Fh = F.cpu().numpy()
    b = -dV.cpu().numpy()
    for w in range(W):
        _, J = oracle.cv_eval(pos[w * n:(w + 1) * n].astype(np.float64), cvs)
        assert rel_inf(Fh[w * n:(w + 1) * n], np.einsum("d,dni->ni", b[w], J)) <= 1e-5
    assert s.abf_grid(0)[0].sum() == Nbefore + 1  # samples keep accumulating
