"""Bias surrogate on the GPU against the FP64 oracle of the network, and
the surrogate step against the exact hill sum.

Parity of the network kernels (oracle on the same bf16-rounded weights,
activations rounded as bf16 hi + lo pairs where the GPU feeds the matrix
cores):
  forward   V, dV/dxi   <= 2e-5 of the batch's largest |y|, |dy| (FP32 math);
            against the oracle with unrounded activations, per sample within
            the first-order bound of the 2^-16 pair rounding plus that 2e-5
  reverse   loss <= 1e-5 relative; gradients <= 1e-4 of each parameter
            block's largest entry (FP32 per-workgroup partials)
  Adam      one and two steps against the update rule on the oracle's
            gradients
Surrogate workload: 100,000 hills of a converged two-CV well-tempered run
(sigma 0.3 rad, w ~ U[0.5, 1.5] kJ/mol, T 300 K, bias factor 6), training on
2^17 torus points, certification on a 512^2 grid at 0.1 kJ/mol/rad, 256
walkers of 22 atoms.  Walkers in certified cells: |dVhat - dV|_2 <= 0.1
against the FP64 hill sum; the others: the exact path's bar (V 1e-6, dV and
forces 1e-5).
"""
import numpy as np
import pytest
import torch

from oracle import _clib as oracle
from oracle import methods, mlp
from paper_2301_04835_amd import synth, synth_wt
from paper_2301_04835_amd.api import Sampler, SxError
from gpu_util import TWO_PI, dev, hill_grad_bound, hill_v_rel_bound, rel_inf

pytestmark = pytest.mark.gpu


def to_dict(v, H, D):
    F = 2 * D
    shapes = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
    out, o = {}, 0
    for k, sh in shapes:
        n = int(np.prod(sh))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(sh)
        o += n
    assert o == len(v)
    return out


def to_flat(P):
    return np.concatenate([np.ravel(P[k]) for k in mlp.PARAM_ORDER]).astype(np.float32)


def rand_params(H, D, seed, scale=0.6):
    g = np.random.default_rng(seed)
    P = mlp.init_params(H, 2 * D, seed)
    for k in P:
        P[k] = P[k] * 2.0 + scale * 0.3 * g.normal(size=P[k].shape)
    return to_flat(P)


def bf16_dict(flat, H, D):
    return {k: mlp.round_bf16(v) for k, v in to_dict(flat, H, D).items()}


def make_ctx(cvs, H, D, max_batch=4096, cert_n=64, K=16, n_atoms=12, walkers=None, shared=False):
    s = Sampler(0)
    s.add_cvs(cvs)
    if walkers is not None:
        s.set_walkers(walkers, [K], shared=shared)
    s.metad([0.3] * D, 1.0, 300.0, None, 0, K)
    s.surrogate(H, max_samples=1 << 17, max_batch=max_batch, cert_n=cert_n, tol_force=0.1)
    s.bind()
    return s


CV_SETS = {
    1: ([{"kind": "dihedral", "idx": [0, 1, 2, 3]}], [True], 64),
    2: (synth.backbone_cvs(0), [True, True], 64),
    3: (synth.backbone_cvs(0) + [{"kind": "gyration", "idx": [0, 1, 2, 3, 4, 5]}], [True, True, False], 128),
}


@pytest.mark.parametrize("D", [1, 2, 3])
def test_forward_matches_oracle(gpu, D):
    cvs, periodic, H = CV_SETS[D]
    s = make_ctx(cvs, H, D)
    mu, sd = np.array([0.0, 0.0, 0.9])[:D], np.array([1.0, 1.0, 0.25])[:D]
    if not all(periodic):
        s.surrogate_norm(mu, sd)
    P = rand_params(H, D, 10 + D)
    assert s.surrogate_param_count() == P.size
    s.surrogate_params(P)
    s.surrogate_output(1.7, 3.0)
    n = 5000
    g = np.random.default_rng(20 + D)
    xi = g.uniform(-np.pi, np.pi, size=(n, D))
    if D == 3:
        xi[:, 2] = 0.9 + 0.3 * g.normal(size=n)
    V, dV = s.surrogate_eval(dev(xi))
    y, dy, _ = mlp.forward(bf16_dict(P, H, D), xi, periodic, mu, sd, act_round=mlp.round_bf16x2)
    Vr, dVr = 3.0 + 1.7 * y, 1.7 * dy
    eV = np.max(np.abs(V.cpu().numpy() - Vr)) / (1.7 * np.max(np.abs(y)))
    edV = max(np.max(np.abs(dV.cpu().numpy()[:, d] - dVr[:, d])) / np.max(np.abs(dVr[:, d])) for d in range(D))
    print(f"D={D} H={H}: V err {eV:.2e}, dV err {edV:.2e}")
    assert eV <= 2e-5 and edV <= 2e-5
    # the bf16 pair rounding of the activations is what the GPU does: single
    # bf16 rounding would be visibly further away
    y1, _, _ = mlp.forward(bf16_dict(P, H, D), xi, periodic, mu, sd, act_round=mlp.round_bf16)
    assert np.max(np.abs(3.0 + 1.7 * y1 - V.cpu().numpy())) > 5 * np.max(np.abs(V.cpu().numpy() - Vr))
    # against the plain FP64 network (the same bf16 weights, activations not
    # rounded): the pair hi + lo carries an activation a to |a - hi - lo| <=
    # 2^-8 |a - hi| <= 2^-16 |a| (bf16 keeps 8 significant bits; a is first
    # rounded to float32), so to first order the rounding moves
    #   y    by <= u sum_i |w3_i| (1 - a2_i^2) sum_j |W2_ij| |a1_j|
    #   dy_d by <= u sum_i |w3_i| [(1 - a2_i^2) sum_j |W2_ij| |da1_dj|
    #                              + 2 |a2_i| |dz2_di| (1 - a2_i^2) sum_j |W2_ij| |a1_j|]
    # with u = 2^-16 + 2^-24; the kernel's FP32 arithmetic adds the 2e-5 above
    Pb = bf16_dict(P, H, D)
    yp, dyp, c = mlp.forward(Pb, xi, periodic, mu, sd)
    u = 2.0 ** -16 + 2.0 ** -24
    W2a, w3a = np.abs(Pb["W2"]), np.abs(Pb["w3"])
    s2 = 1.0 - c["a2"] ** 2
    za = np.abs(c["a1"]) @ W2a.T
    by = u * (s2 * za) @ w3a
    errV = np.abs(V.cpu().numpy() - (3.0 + 1.7 * yp))
    assert np.all(errV <= 1.7 * (1.01 * by + 2e-5 * np.max(np.abs(y)))), np.max(errV / (1.7 * by))
    for d in range(D):
        zd = np.abs(c["da1"][d]) @ W2a.T
        bdy = u * (s2 * zd + 2.0 * np.abs(c["a2"]) * np.abs(c["dz2"][d]) * s2 * za) @ w3a
        errd = np.abs(dV.cpu().numpy()[:, d] - 1.7 * dyp[:, d])
        assert np.all(errd <= 1.7 * (1.01 * bdy + 2e-5 * np.max(np.abs(dy[:, d])))), (d, np.max(errd / (1.7 * bdy)))
    print(f"D={D} H={H}: vs the unrounded network, largest error / derived bound: V "
          f"{np.max(errV / (1.7 * by)):.2f}")


@pytest.mark.parametrize("D", [2, 3])
def test_loss_gradients_match_oracle(gpu, D):
    cvs, periodic, H = CV_SETS[D]
    s = make_ctx(cvs, H, D)
    mu, sd = np.array([0.0, 0.0, 0.9])[:D], np.array([1.0, 1.0, 0.25])[:D]
    if not all(periodic):
        s.surrogate_norm(mu, sd)
    P = rand_params(H, D, 30 + D)
    s.surrogate_params(P)
    s.surrogate_output(1.5, 0.5)
    n = 4096
    g = np.random.default_rng(40 + D)
    xi = g.uniform(-np.pi, np.pi, size=(n, D))
    if D == 3:
        xi[:, 2] = 0.9 + 0.3 * g.normal(size=n)
    V = 2.0 + 3.0 * g.normal(size=n)
    G = 2.0 * g.normal(size=(n, D))
    loss, grad = s.surrogate_loss_grad(dev(xi), dev(V), dev(G), 0.7, 1.3)
    L, gr, _, _ = mlp.loss_and_grads(bf16_dict(P, H, D), xi, (V - 0.5) / 1.5, G / 1.5, 0.7, 1.3, periodic, mu, sd,
                                     act_round=mlp.round_bf16x2)
    gk = to_dict(grad, H, D)
    assert abs(loss - L) <= 1e-5 * L
    worst = {k: np.max(np.abs(gk[k] - gr[k])) / np.max(np.abs(gr[k])) for k in gr}
    print(f"D={D} H={H}: loss {loss:.6g} vs {L:.6g}; gradient errors", {k: f"{v:.1e}" for k, v in worst.items()})
    assert max(worst.values()) <= 1e-4


def test_adam_steps_match_update_rule(gpu):
    cvs, periodic, H = CV_SETS[2]
    D = 2
    s = make_ctx(cvs, H, D)
    P0 = rand_params(H, D, 50)
    s.surrogate_params(P0)
    n = 2048
    g = np.random.default_rng(51)
    xi = g.uniform(-np.pi, np.pi, size=(n, D))
    V, G = g.normal(size=n), g.normal(size=(n, D))
    lr = 1e-3
    s.surrogate_fit(dev(xi), dev(V), dev(G), batch=n, steps=1, lr=lr, lr_final=lr, alpha=1.0, beta=0.5)
    P1 = s.surrogate_params()
    _, g1, _, _ = mlp.loss_and_grads(bf16_dict(P0, H, D), xi, V, G, 1.0, 0.5, periodic, act_round=mlp.round_bf16x2)
    zero = {k: np.zeros_like(v) for k, v in g1.items()}
    R1, m1, v1 = mlp.adam_step(to_dict(P0, H, D), g1, zero, zero, 1, lr)
    p1 = to_dict(P1, H, D)
    for k in g1:
        big = np.abs(g1[k]) > 1e-3 * np.max(np.abs(g1[k]))
        # t = 1 moves every parameter by lr sign(g) (up to eps)
        assert np.max(np.abs(p1[k] - R1[k])[big]) <= 1e-4 * lr + 2e-7 * np.max(np.abs(R1[k])), k
        assert np.all(np.abs(p1[k] - to_dict(P0, H, D)[k]) <= lr * (1 + 1e-6) + 1e-7)
    s.surrogate_fit(dev(xi), dev(V), dev(G), batch=n, steps=1, lr=lr, lr_final=lr, alpha=1.0, beta=0.5)
    P2 = to_dict(s.surrogate_params(), H, D)
    _, g2, _, _ = mlp.loss_and_grads(bf16_dict(P1, H, D), xi, V, G, 1.0, 0.5, periodic, act_round=mlp.round_bf16x2)
    R2, _, _ = mlp.adam_step(p1, g2, m1, v1, 2, lr)
    for k in g2:
        m = 0.9 * m1[k] + 0.1 * g2[k]
        ok = np.abs(m) > 1e-3 * np.max(np.abs(m))
        assert np.max(np.abs(P2[k] - R2[k])[ok]) <= 1e-3 * lr + 2e-7 * np.max(np.abs(R2[k])), k


# ------------------------------------------------------ surrogate workload
K_C4, W_C4 = 100000, 256


@pytest.fixture(scope="module")
def c4(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    C, H = synth_wt.wt_hills(K_C4)
    pos, off = synth.chain_walkers(W_C4, 22, seed=4)
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(4))
    s.set_walkers(off, [K_C4], shared=True)
    s.metad([0.3, 0.3], 1.0, 300.0, 6.0, 0, K_C4)
    s.surrogate(64, max_samples=1 << 17, max_batch=4096, cert_n=512, tol_force=0.1)
    s.bind()
    s.hills_set(0, C, H)
    P0 = to_flat(mlp.init_params(64, 4, 7))
    s.surrogate_params(P0)
    frac0 = s.surrogate_certify()
    X = synth_wt.torus_points(1 << 17, 8)
    loss = s.surrogate_train(dev(X), batch=4096, steps=100000, lr=3e-3, lr_final=1e-5)
    frac = s.surrogate_certify()
    print(f"surrogate: loss {loss:.3e}, certified fraction untrained {frac0:.3f} -> trained {frac:.3f}")
    return dict(s=s, C=C.astype(np.float64), H=H.astype(np.float64), pos=pos, off=off, frac0=frac0, frac=frac)


def test_training_gains_certified_cells(c4):
    assert c4["frac0"] <= 0.01
    assert c4["frac"] >= 0.6


def test_certified_cells_hold_the_force_bound(c4):
    s = c4["s"]
    X = synth_wt.torus_points(20000, 99)
    V, dV, fb = s.surrogate_eval(dev(X), fallback=True)
    fb = fb.cpu().numpy().astype(bool)
    cert = ~fb
    assert cert.sum() > 1000
    Vr, dVr = oracle.hillsum_batch(X[cert], None, c4["C"], c4["H"], [0.3, 0.3], [TWO_PI] * 2, nthreads=8)
    err = np.linalg.norm(dV.cpu().numpy()[cert] - dVr, axis=1)
    print(f"certified points {cert.sum()}: force error max {err.max():.4f}, median {np.median(err):.4f} kJ/mol/rad")
    assert err.max() <= 0.1


def test_surrogate_step_against_exact(c4):
    s = c4["s"]
    pos, off = c4["pos"], c4["off"]
    P = dev(pos)
    s.surrogate_enable(True)
    F = torch.zeros_like(P)
    xi = torch.empty((W_C4, 2), dtype=torch.float64, device=P.device)
    V = torch.empty(W_C4, dtype=torch.float64, device=P.device)
    dV = torch.empty((W_C4, 2), dtype=torch.float64, device=P.device)
    s.step(P, forces=F, step=7, xi_out=xi, V_out=V, dV_out=dV)
    nfb = s.surrogate_fallback_count()
    s.check()
    xi, V, dV, F = (t.cpu().numpy() for t in (xi, V, dV, F))
    Vn, dVn, fb = s.surrogate_eval(dev(xi), fallback=True)
    fb = fb.cpu().numpy().astype(bool)
    assert nfb == fb.sum()
    assert 0 < nfb < W_C4
    Vr, dVr = oracle.hillsum_batch(xi, None, c4["C"], c4["H"], [0.3, 0.3], [TWO_PI] * 2, nthreads=8)
    net = ~fb
    # network walkers: the network's values, within the certified bound of the exact bias
    assert np.array_equal(V[net], Vn.cpu().numpy()[net]) and np.array_equal(dV[net], dVn.cpu().numpy()[net])
    assert np.max(np.linalg.norm(dV[net] - dVr[net], axis=1)) <= 0.1
    # fallback walkers: the exact path's bar
    assert np.max(np.abs(V[fb] - Vr[fb]) / np.abs(Vr[fb])) <= 1e-6
    assert max(rel_inf(dV[w], dVr[w]) for w in np.where(fb)[0]) <= 1e-5
    # forces are the chain rule of whichever dV/dxi the walker used
    cvs = synth.backbone_cvs(4)
    for w in range(W_C4):
        x = pos[off[w]:off[w + 1]].astype(np.float64)
        xr, J = methods.cv_eval(x, cvs, None)
        assert np.max(np.abs(xr - xi[w])) <= 1e-6
        assert rel_inf(F[off[w]:off[w + 1]], methods.chain_rule(-dV[w], J)) <= 1e-5
    # nothing deposited; the step counter moved
    assert s.hills_get(0)[0].shape[0] == len(c4["H"])
    assert s.get_step() == 8
    # graph replay of surrogate steps reproduces the eager step
    F2 = torch.zeros_like(P)
    xo = torch.empty((W_C4, 2), dtype=torch.float64, device=P.device)
    Vo = torch.empty(W_C4, dtype=torch.float64, device=P.device)
    s.graph_capture(3, P, forces=F2, xi_out=xo, V_out=Vo)
    for _ in range(2):
        s.graph_launch()
        torch.cuda.synchronize()
        assert np.array_equal(Vo.cpu().numpy(), V)
    assert np.allclose(F2.cpu().numpy(), 6 * F, rtol=1e-6, atol=1e-6)
    s.surrogate_enable(False)


@pytest.mark.parametrize("W", [8, 40, 1100])
def test_fallback_with_spare_capacity(gpu, W):
    """A shared list filled to a fraction of its capacity (3,000 hills in
    room for 15,000: the fallback sums' chunks past the count hold no
    hills) and an untrained network that certifies nothing, so every walker
    takes the exact fallback, right after a certification pass has left
    other records in the same workspace: V and dV/dxi of every walker
    against the oracle at the derived bounds of an FP32-term hill sum.  8
    walkers: one per workgroup row of the fallback grid; 40: rows that sum
    two walkers from the same loaded chunk; 1,100: more walkers than the
    compacted grid serves, one row per walker."""
    K, cap = 3000, 15000
    C = synth.uniform_centers(K, 2, 41)
    H = synth.uniform_heights(K, 42)
    pos, off = synth.chain_walkers(W, 22, seed=43)
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(4))
    s.set_walkers(off, [cap], shared=True)
    s.metad([0.3, 0.3], 1.0, 300.0, 6.0, 0, cap)
    s.surrogate(64, max_samples=1024, max_batch=2048, cert_n=32, tol_force=0.1)
    s.bind()
    s.hills_set(0, C, H)
    s.surrogate_params(rand_params(64, 2, 44))
    s.surrogate_certify()
    s.surrogate_enable(True)
    P = dev(pos)
    F = torch.zeros_like(P)
    xi = torch.empty((W, 2), dtype=torch.float64, device=P.device)
    V = torch.empty(W, dtype=torch.float64, device=P.device)
    dV = torch.empty((W, 2), dtype=torch.float64, device=P.device)
    s.step(P, forces=F, step=3, xi_out=xi, V_out=V, dV_out=dV)
    s.check()
    assert s.surrogate_fallback_count() == W
    xi, V, dV = (t.cpu().numpy() for t in (xi, V, dV))
    Cd, Hd = C.astype(np.float64), H.astype(np.float64)
    Vr, dVr = oracle.hillsum_batch(xi, None, Cd, Hd, [0.3, 0.3], [TWO_PI] * 2, nthreads=8)
    per, zero = [TWO_PI] * 2, np.zeros((2, 2))
    for w in range(W):
        assert abs(V[w] - Vr[w]) <= hill_v_rel_bound(xi[w], Cd, Hd, [0.3, 0.3], per) * abs(Vr[w])
        assert np.all(np.abs(dV[w] - dVr[w]) <= hill_grad_bound(xi[w], Cd, Hd, [0.3, 0.3], per, zero, np.zeros(2)))


def test_surrogate_errors(gpu):
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(0))
    with pytest.raises(SxError) as e:
        s.surrogate(32)
    assert e.value.status == 1
    s.metad([0.3, 0.3], 1.0, 300.0, None, 0, 64)
    s.surrogate(64, max_samples=1024, max_batch=256, cert_n=16)
    s.bind()
    with pytest.raises(SxError) as e:
        s.surrogate_enable(True)
    assert e.value.status == 6
    s.surrogate_params(rand_params(64, 2, 1))
    xi = dev(np.zeros((4, 2)))
    with pytest.raises(SxError) as e:
        s.surrogate_eval(xi, fallback=True)
    assert e.value.status == 6
    with pytest.raises(SxError) as e:
        s.surrogate_loss_grad(dev(np.zeros((512, 2))), dev(np.zeros(512)), dev(np.zeros((512, 2))), 1.0, 1.0)
    assert e.value.status == 1
    # private lists of several walkers cannot share one network
    p = Sampler(0)
    p.add_cvs(synth.backbone_cvs(0))
    p.set_walkers([0, 12, 24], [16, 16])
    p.metad([0.3, 0.3], 1.0, 300.0, None, 0, 16)
    p.surrogate(64, max_samples=1024, max_batch=256, cert_n=16)
    p.bind()
    p.surrogate_params(rand_params(64, 2, 2))
    p.surrogate_certify()
    with pytest.raises(SxError) as e:
        p.surrogate_enable(True)
    assert e.value.status == 6
