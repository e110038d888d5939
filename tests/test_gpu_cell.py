"""Coordination numbers through cell lists against the FP64 oracle (brute
force over all pairs with the minimum image and the hard cut).

  CN values    <= 1e-6 relative (FP32 pair terms relative to cell origins,
               FP64 sums)
  VJP / forces <= 1e-5 relative (inf-norm over a walker's atoms)
"""
import numpy as np
import pytest
import torch

from oracle import _clib as oracle
from oracle import methods
from paper_2301_04835_amd import synth
from paper_2301_04835_amd.api import Sampler, SxError
from gpu_util import dev, rel_inf

pytestmark = pytest.mark.gpu


def small_system(W, n, L, seed, self_cn=False):
    """Three groups of n atoms per walker, some outside [0, L) and some
    exactly on cell faces (cells of L / 3)."""
    g = np.random.default_rng(seed)
    pos = g.uniform(0.0, L, size=(W * 3 * n, 3))
    pos[::7] += g.choice([-L, L, 2 * L], size=(pos[::7].shape[0], 1))  # outside the box: wrapped
    pos[3::11, 0] = L / 3.0                                            # on a cell face
    pos[5::13, 1] = 0.0
    pos[6::17, 2] = L                                                  # on the far face = 0
    off = np.arange(W + 1, dtype=np.int64) * 3 * n
    cvs = synth.cn3_cvs(n, 0.5, 1.2)
    if self_cn:  # one group with itself: i == j skipped, the gradient counts both sides
        cvs.append({"kind": "coordination", "a": list(range(n)), "b": list(range(n)), "r0": 0.45, "n": 8,
                    "m": 14, "rcut": 1.1, "normalize": False})
    return pos.astype(np.float32), off, cvs


def oracle_walker(pos_w, cvs, L):
    xi, J = methods.cv_eval(pos_w.astype(np.float64), cvs, np.full(3, L))
    return xi, J


def ctx(cvs, L, off, mode, metad=None):
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_box([L, L, L])
    s.set_walkers(off, metad["cap"] if metad else None, shared=bool(metad))
    s.set_cell_lists(mode)
    if metad:
        s.metad([metad["sigma"]] * len(cvs), 1.0, 300.0, 6.0, 0, metad["cap"])
    s.bind()
    return s


@pytest.mark.parametrize("self_cn", [False, True])
def test_cell_values_and_vjp_against_oracle(gpu, self_cn):
    W, n, L = 3, 700, 4.0
    pos, off, cvs = small_system(W, n, L, 21, self_cn)
    s = ctx(cvs, L, off, 1)
    assert s.cell_list_cvs() == len(cvs)
    P = dev(pos)
    xi = s.eval_cv(P)[0].cpu().numpy()
    g = np.random.default_rng(3)
    xb = g.normal(size=(W, len(cvs)))
    pb = torch.zeros_like(P)
    s.cv_vjp(P, dev(xb), pb)
    pb = pb.cpu().numpy()
    # the all-pairs kernels on the same input
    a = ctx(cvs, L, off, -1)
    assert a.cell_list_cvs() == 0
    xa = a.eval_cv(P)[0].cpu().numpy()
    for w in range(W):
        pw = pos[off[w]:off[w + 1]]
        xr, J = oracle_walker(pw, cvs, L)
        assert np.max(np.abs(xi[w] - xr) / np.abs(xr)) <= 1e-6
        assert np.max(np.abs(xa[w] - xr) / np.abs(xr)) <= 1e-6
        ref = np.tensordot(xb[w], J, axes=1)
        assert rel_inf(pb[off[w]:off[w + 1]], ref) <= 1e-5


def test_cell_values_dense_groups_several_staging_rounds(gpu):
    """Groups of 2,000 in a 4 nm box (31 atoms per nm^3): a column block's
    partner region holds ~3,300 members, more than one LDS staging round
    (1,536), so the pair pass restages and adds later rounds to the earlier
    ones; values and VJP against the brute-force oracle."""
    W, n, L = 2, 2000, 4.0
    pos, off, cvs = small_system(W, n, L, 22)
    s = ctx(cvs, L, off, 1)
    assert s.cell_list_cvs() == 3
    P = dev(pos)
    xi = s.eval_cv(P)[0].cpu().numpy()
    xb = np.random.default_rng(4).normal(size=(W, 3))
    pb = torch.zeros_like(P)
    s.cv_vjp(P, dev(xb), pb)
    pb = pb.cpu().numpy()
    for w in range(W):
        xr, J = oracle_walker(pos[off[w]:off[w + 1]], cvs, L)
        assert np.max(np.abs(xi[w] - xr) / np.abs(xr)) <= 1e-6
        assert rel_inf(pb[off[w]:off[w + 1]], np.tensordot(xb[w], J, axes=1)) <= 1e-5


def test_cell_results_repeat_bitwise(gpu):
    """The build places each member by its rank in member order among its
    cell's members, whatever order the cell slots were taken in: repeated
    evaluations of the dense system (~19 members per sub-cell) give bitwise the
    same CN values and VJP."""
    W, n, L = 2, 2000, 4.0
    pos, off, cvs = small_system(W, n, L, 27)
    s = ctx(cvs, L, off, 1)
    P = dev(pos)
    xb = dev(np.random.default_rng(5).normal(size=(W, 3)))
    runs = []
    for _ in range(3):
        xi = s.eval_cv(P)[0].cpu().numpy()
        pb = torch.zeros_like(P)
        s.cv_vjp(P, xb, pb)
        runs.append((xi, pb.cpu().numpy()))
    for xi, pb in runs[1:]:
        assert np.array_equal(xi, runs[0][0]) and np.array_equal(pb, runs[0][1])


@pytest.mark.parametrize("mode", [1, -1])
def test_cut_edge_decisions_match_oracle(gpu, mode):
    """Pairs placed at the hard cut, r = rcut (1 + delta) for delta from
    -3e-5 to 3e-5 (the FP32 float positions move each by ~2e-7 relative),
    some across the periodic boundary: every pair must fall on the side the
    FP64 definition puts it (inside unless r >= rcut, from the positions as
    given), through the cell lists (mode 1) and all pairs (mode -1).  One
    pair decided the other way moves the unnormalised CN by s(rcut) = 5.2e-3;
    the test allows a fifth of that."""
    W, na, L, rc = 2, 64, 4.0, 1.2
    deltas = np.array([-3e-5, -8e-6, -2e-6, -2e-7, -1e-8, 1e-8, 2e-7, 2e-6, 8e-6, 3e-5])
    g = np.random.default_rng(28)
    blocks = []
    for w in range(W):
        a = g.uniform(0.0, L, size=(na, 3))
        u = g.normal(size=(na, deltas.size, 3))
        u /= np.linalg.norm(u, axis=2, keepdims=True)
        b = (a[:, None, :] + rc * (1.0 + deltas)[None, :, None] * u).reshape(-1, 3)
        blocks.append(np.concatenate([a, np.mod(b, L)]))  # partners wrapped into the box
    pos = np.concatenate(blocks).astype(np.float32)
    n = na * (1 + deltas.size)
    off = np.arange(W + 1, dtype=np.int64) * n
    cvs = [{"kind": "coordination", "a": list(range(na)), "b": list(range(na, n)), "r0": 0.5, "n": 6, "m": 12,
            "rcut": rc, "normalize": False}]
    s = ctx(cvs, L, off, mode)
    assert s.cell_list_cvs() == (1 if mode == 1 else 0)
    P = dev(pos)
    xi = s.eval_cv(P)[0].cpu().numpy()
    xb = np.random.default_rng(29).normal(size=(W, 1))
    pb = torch.zeros_like(P)
    s.cv_vjp(P, dev(xb), pb)
    pb = pb.cpu().numpy()
    s_cut = 1.0 / (1.0 + (rc / 0.5) ** 6)
    for w in range(W):
        pw = pos[off[w]:off[w + 1]]
        xr, J = oracle_walker(pw, cvs, L)
        d = pw[na:].astype(np.float64).reshape(na, deltas.size, 3) - pw[:na, None, :].astype(np.float64)
        d -= L * np.rint(d / L)
        r = np.sqrt(np.sum(d * d, axis=2))
        assert np.sum(r < rc) > 0 and np.sum(r >= rc) > 0  # both sides of the cut are present
        assert abs(xi[w, 0] - xr[0]) <= 0.2 * s_cut
        assert rel_inf(pb[off[w]:off[w + 1]], np.tensordot(xb[w], J, axes=1)) <= 1e-5


def test_cell_values_orthorhombic_box(gpu):
    """An orthorhombic box with a different cell count per dimension
    (4.0 x 5.3 x 7.9 nm: 3, 4 and 6 cut-length cells, z cut further into
    sub-cells), atoms outside the box and on cell faces: values and VJP
    against the brute-force oracle with the same box."""
    W, n = 2, 600
    box = np.array([4.0, 5.3, 7.9])
    g = np.random.default_rng(25)
    pos = g.uniform(0.0, 1.0, size=(W * 3 * n, 3)) * box
    pos[::7] += g.choice([-1.0, 1.0, 2.0], size=(pos[::7].shape[0], 1)) * box  # wrapped
    pos[3::11, 1] = box[1] / 4.0  # on a cell face
    pos[5::13, 2] = box[2]        # on the far face = 0
    pos = pos.astype(np.float32)
    off = np.arange(W + 1, dtype=np.int64) * 3 * n
    cvs = synth.cn3_cvs(n, 0.5, 1.2)
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_box(list(box))
    s.set_walkers(off)
    s.set_cell_lists(1)
    s.bind()
    assert s.cell_list_cvs() == 3
    P = dev(pos)
    xi = s.eval_cv(P)[0].cpu().numpy()
    xb = np.random.default_rng(26).normal(size=(W, 3))
    pb = torch.zeros_like(P)
    s.cv_vjp(P, dev(xb), pb)
    pb = pb.cpu().numpy()
    for w in range(W):
        xr, J = methods.cv_eval(pos[off[w]:off[w + 1]].astype(np.float64), cvs, box)
        assert np.max(np.abs(xi[w] - xr) / np.abs(xr)) <= 1e-6
        assert rel_inf(pb[off[w]:off[w + 1]], np.tensordot(xb[w], J, axes=1)) <= 1e-5


def test_cell_mode_rules(gpu):
    W, n, L = 2, 300, 4.0
    pos, off, cvs = small_system(W, n, L, 5)
    # default mode: groups this small stay on the all-pairs kernels
    assert ctx(cvs, L, off, 0).cell_list_cvs() == 0
    # a box narrower than three cutoffs cannot use cells
    assert ctx(cvs, 3.3, off, 1).cell_list_cvs() == 0
    # groups that overlap without being identical are refused in mode 1
    bad = [dict(cvs[0]), dict(cvs[1])]
    bad[1]["a"] = list(range(n // 2, n + n // 2))
    s = Sampler(0)
    s.add_cvs(bad)
    s.set_box([L, L, L])
    s.set_walkers(off)
    s.set_cell_lists(1)
    with pytest.raises(SxError) as e:
        s.bind()
    assert e.value.status == 1


def test_cell_step_shared_hills_3d(gpu):
    """Metadynamics step: three cell-list CNs, a shared list of 3-D hills,
    forces from the VJP kernel, against the oracle's chain rule."""
    W, n, L, K = 4, 800, 4.0, 5000
    pos, off, cvs = small_system(W, n, L, 8)
    P = dev(pos)
    s = ctx(cvs, L, off, 1, {"sigma": 0.2, "cap": K + 4 * W})
    xi0 = s.eval_cv(P)[0].cpu().numpy()
    g = np.random.default_rng(9)
    C = (xi0.mean(axis=0) + 0.3 * g.normal(size=(K, 3))).astype(np.float32)
    H = g.uniform(0.5, 1.5, size=K).astype(np.float32)
    s.hills_set(0, C, H)
    F = torch.zeros_like(P)
    xi = torch.zeros((W, 3), dtype=torch.float64, device=P.device)
    V = torch.zeros(W, dtype=torch.float64, device=P.device)
    dV = torch.zeros((W, 3), dtype=torch.float64, device=P.device)
    s.step(P, forces=F, step=1, xi_out=xi, V_out=V, dV_out=dV)
    s.check()
    xi, V, dV, F = (t.cpu().numpy() for t in (xi, V, dV, F))
    Vr, dVr = oracle.hillsum_batch(xi, None, C.astype(np.float64), H.astype(np.float64), [0.2] * 3, [0.0] * 3,
                                   nthreads=8)
    assert np.max(np.abs(V - Vr) / Vr) <= 1e-6
    for w in range(W):
        assert rel_inf(dV[w], dVr[w]) <= 1e-5
        xr, J = oracle_walker(pos[off[w]:off[w + 1]], cvs, L)
        assert np.max(np.abs(xi[w] - xr) / xr) <= 1e-6
        assert rel_inf(F[off[w]:off[w + 1]], methods.chain_rule(-dV[w], J)) <= 1e-5


def test_cn3_full_size_sampled(gpu):
    """512 walkers of 60,000 atoms in a 12 nm box, groups of 20,000 (default
    mode picks the cell lists); walker 137 checked against the oracle."""
    p = synth.CN3
    W, n = 512, p["n_group"]
    cvs = synth.cn3_cvs(n, p["r0"], p["rcut"])
    pos, off = synth.cn3_positions(W, n, p["box"])
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_box([p["box"]] * 3)
    s.set_walkers(off)
    s.bind()
    assert s.cell_list_cvs() == 3
    P = dev(pos)
    xi = s.eval_cv(P)[0].cpu().numpy()
    assert np.all(np.abs(xi - p["cn_mean"]) < 0.2)
    w = 137
    xb = np.zeros((W, 3))
    xb[w] = [0.7, -1.3, 0.4]
    pb = torch.zeros_like(P)
    s.cv_vjp(P, dev(xb), pb)
    xr, J = oracle_walker(pos[off[w]:off[w + 1]], cvs, p["box"])
    assert np.max(np.abs(xi[w] - xr) / xr) <= 1e-6
    pbw = pb.cpu().numpy()
    assert rel_inf(pbw[off[w]:off[w + 1]], np.tensordot(xb[w], J, axes=1)) <= 1e-5
    assert np.all(pbw[:off[w]] == 0) and np.all(pbw[off[w + 1]:] == 0)


def test_cn3_full_size_step_sampled_walkers(gpu):
    """The full-size step: 512 walkers of 60,000 atoms, three cell-list CNs
    over 20,000-atom groups, one shared list of 10^6 three-dimensional hills
    (sigma 0.2, centres around the expected CN), the forces as the VJP of
    dV/dxi, as the benchmark runs it.  Eight walkers spread over the batch
    against the oracle (brute force over all pairs for xi and J, the FP64
    hill sum over the 10^6 hills at the oracle's xi): xi 1e-6, V within its
    float32-term bound; dV/dxi and the forces within their derived bounds:
    the walkers sit inside the hill cloud, where dV/dxi is a small remainder
    of large terms of both signs and the bias is steep, so the bound is 1e-5
    of the term scale (the sum of the terms' magnitudes) plus what the
    CV tolerance of 1e-6 moves the gradient through the oracle's Hessian
    (central differences); the forces add J's 1e-5.  Every walker's V finite
    and positive, and every walker's V and dV/dxi within the same bounds of
    the oracle's hill sum taken at the GPU's own xi."""
    import concurrent.futures as cf

    from gpu_util import hill_grad_bound, hill_v_rel_bound

    p = synth.CN3
    W, n, K = 512, p["n_group"], 1000000
    cvs = synth.cn3_cvs(n, p["r0"], p["rcut"])
    pos, off = synth.cn3_positions(W, n, p["box"])
    C, H = synth.cn3_hills(K, mean=p["cn_mean"], sd=p["hill_sd"])
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_box([p["box"]] * 3)
    s.set_walkers(off, [K + 64 * W], shared=True)
    s.metad([p["sigma"]] * 3, 1.0, 300.0, 6.0, 0, K + 64 * W)
    s.bind()
    assert s.cell_list_cvs() == 3
    s.hills_set(0, C, H)
    P = dev(pos)
    F = torch.zeros_like(P)
    xi = torch.zeros((W, 3), dtype=torch.float64, device=gpu)
    V = torch.zeros(W, dtype=torch.float64, device=gpu)
    dV = torch.zeros((W, 3), dtype=torch.float64, device=gpu)
    s.step(P, forces=F, step=1, xi_out=xi, V_out=V, dV_out=dV)
    s.check()
    xi, V, dV, F = (t.cpu().numpy() for t in (xi, V, dV, F))
    assert np.all(np.isfinite(V)) and np.all(V > 0)
    ws = [0, 73, 146, 219, 292, 365, 438, 511]
    with cf.ThreadPoolExecutor(8) as ex:
        ref = list(ex.map(lambda w: oracle_walker(pos[off[w]:off[w + 1]], cvs, p["box"]), ws))
    xr = np.array([r[0] for r in ref])
    Cd, Hd, sig, per = C.astype(np.float64), H.astype(np.float64), [p["sigma"]] * 3, [0.0] * 3
    Vr, dVr = oracle.hillsum_batch(xr, None, Cd, Hd, sig, per, nthreads=8)
    # the oracle's Hessian of V at its xi: central differences of dV/dxi
    hstep = 1e-4
    shifts = np.concatenate([xr[:, None, :] + hstep * s_ * np.eye(3)[None] for s_ in (1.0, -1.0)], axis=1)
    _, dVs = oracle.hillsum_batch(shifts.reshape(-1, 3), None, Cd, Hd, sig, per, nthreads=8)
    dVs = dVs.reshape(len(ws), 6, 3)
    hess = (dVs[:, :3, :] - dVs[:, 3:, :]).transpose(0, 2, 1) / (2 * hstep)  # [w][d][e] = d2V/dxi_d dxi_e
    worst = {"xi": 0.0, "V/bound": 0.0, "dV/bound": 0.0, "F/bound": 0.0, "dV_rel": 0.0, "F_rel": 0.0}
    for i, w in enumerate(ws):
        worst["xi"] = max(worst["xi"], np.max(np.abs(xi[w] - xr[i]) / xr[i]))
        bV = hill_v_rel_bound(xr[i], C, H, sig, per)
        worst["V/bound"] = max(worst["V/bound"], abs(V[w] - Vr[i]) / Vr[i] / bV)
        bdV = hill_grad_bound(xr[i], C, H, sig, per, hess[i], 1e-6 * np.abs(xr[i]))
        worst["dV/bound"] = max(worst["dV/bound"], np.max(np.abs(dV[w] - dVr[i]) / bdV))
        J = ref[i][1]
        Fr = methods.chain_rule(-dVr[i], J)
        bF = np.sum((bdV + 1e-5 * np.abs(dVr[i])) * np.max(np.abs(J), axis=(1, 2)))
        worst["F/bound"] = max(worst["F/bound"], np.max(np.abs(F[off[w]:off[w + 1]] - Fr)) / bF)
        worst["dV_rel"] = max(worst["dV_rel"], rel_inf(dV[w], dVr[i]))
        worst["F_rel"] = max(worst["F_rel"], rel_inf(F[off[w]:off[w + 1]], Fr))
    print("worst over the sampled walkers:", worst)
    assert worst["xi"] <= 1e-6 and worst["V/bound"] <= 1.0
    assert worst["dV/bound"] <= 1.0 and worst["F/bound"] <= 1.0
    # every walker's V and dV/dxi against the oracle's hill sum over the 10^6
    # hills at the GPU's own xi (the CV tolerance then does not enter): V
    # within its float32-term bound, dV/dxi within 1e-5 of its term scale
    Vg, dVg = oracle.hillsum_batch(xi, None, Cd, Hd, sig, per, nthreads=16)
    zero3, nil = np.zeros((3, 3)), np.zeros(3)
    with cf.ThreadPoolExecutor(16) as ex:
        bnd = list(ex.map(lambda w: (hill_v_rel_bound(xi[w], Cd, Hd, sig, per),
                                     hill_grad_bound(xi[w], Cd, Hd, sig, per, zero3, nil)), range(W)))
    rV = max(abs(V[w] - Vg[w]) / Vg[w] / bnd[w][0] for w in range(W))
    rdV = max(np.max(np.abs(dV[w] - dVg[w]) / bnd[w][1]) for w in range(W))
    print("all %d walkers at the GPU's xi: V err / bound %.3f, dV err / bound %.3f" % (W, rV, rdV))
    assert rV <= 1.0 and rdV <= 1.0


def test_cell_surrogate_step(gpu):
    """Surrogate on three cell-list CNs (6-128-128-1 on standardised CNs):
    each walker gets the network's or the exact bias by its cell's
    certification, and its forces are the VJP of the dV/dxi it got."""
    W, n, L, K = 6, 800, 4.0, 3000
    pos, off, cvs = small_system(W, n, L, 30)
    P = dev(pos)
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_box([L, L, L])
    s.set_walkers(off, [K + 64], shared=True)
    s.set_cell_lists(1)
    s.metad([0.2] * 3, 1.0, 300.0, 6.0, 0, K + 64)
    s.surrogate(128, max_samples=1 << 14, max_batch=1024, cert_n=24, tol_force=1.0)
    s.bind()
    xi0 = s.eval_cv(P)[0].cpu().numpy()
    mu, sd = xi0.mean(axis=0), 0.3
    g = np.random.default_rng(31)
    C = (mu + sd * g.normal(size=(K, 3))).astype(np.float32)
    H = g.uniform(0.5, 1.5, size=K).astype(np.float32)
    s.hills_set(0, C, H)
    s.surrogate_norm(mu, [sd] * 3)
    P0 = np.concatenate([np.ravel(v) for v in mlp_init(128, 6)]).astype(np.float32)
    s.surrogate_params(P0)
    X = dev(mu + sd * g.normal(size=(1 << 14, 3)))
    s.surrogate_train(X, batch=1024, steps=3000, lr=3e-3, lr_final=1e-5)
    _, dVx = s.bias_eval(X[:2048])
    s.surrogate_tolerance(0.05 * float(torch.sqrt((dVx ** 2).sum(1).mean()).item()))
    frac = s.surrogate_certify(mu - 1.0, mu + 1.0)
    assert 0.0 < frac < 1.0
    s.surrogate_enable(True)
    F = torch.zeros_like(P)
    xi = torch.zeros((W, 3), dtype=torch.float64, device=P.device)
    V = torch.zeros(W, dtype=torch.float64, device=P.device)
    dV = torch.zeros((W, 3), dtype=torch.float64, device=P.device)
    s.step(P, forces=F, step=0, xi_out=xi, V_out=V, dV_out=dV)
    s.check()
    Vn, dVn, fb = s.surrogate_eval(xi, fallback=True)
    fb = fb.cpu().numpy().astype(bool)
    xi, V, dV, F = (t.cpu().numpy() for t in (xi, V, dV, F))
    assert s.surrogate_fallback_count() == fb.sum()
    Vr, dVr = oracle.hillsum_batch(xi, None, C.astype(np.float64), H.astype(np.float64), [0.2] * 3, [0.0] * 3,
                                   nthreads=8)
    for w in range(W):
        if fb[w]:
            assert abs(V[w] - Vr[w]) <= 1e-6 * abs(Vr[w]) and rel_inf(dV[w], dVr[w]) <= 1e-5
        else:
            assert V[w] == Vn.cpu().numpy()[w] and np.array_equal(dV[w], dVn.cpu().numpy()[w])
        xr, J = oracle_walker(pos[off[w]:off[w + 1]], cvs, L)
        assert np.max(np.abs(xi[w] - xr) / xr) <= 1e-6
        assert rel_inf(F[off[w]:off[w + 1]], methods.chain_rule(-dV[w], J)) <= 1e-5


def mlp_init(H, F):
    from oracle import mlp
    P = mlp.init_params(H, F, 2)
    return [P[k] for k in mlp.PARAM_ORDER]


def test_cell_autograd_harmonic(gpu):
    """A harmonic bias k/2 (xi - xi0)^2 on the three cell-list CNs through
    torch.autograd (CVFunction: forward = the cell-list kernels, backward =
    the stored-gradient VJP), against the exact chain rule with the oracle's
    Jacobian, two walkers."""
    from paper_2301_04835_amd.autograd import cv

    W, n, L = 2, 300, 4.0
    pos, off, cvs = small_system(W, n, L, 31)
    s = ctx(cvs, L, off, 1)
    assert s.cell_list_cvs() == 3
    k = torch.tensor([40.0, 25.0, 60.0], dtype=torch.float64, device=gpu)
    xi0 = torch.tensor([1.0, 1.3, 0.8], dtype=torch.float64, device=gpu)
    P = dev(pos).requires_grad_(True)
    xi = cv(P, s)
    (0.5 * (k * (xi - xi0) ** 2)).sum().backward()
    g = P.grad.cpu().numpy()
    for w in range(W):
        xr, J = oracle_walker(pos[off[w]:off[w + 1]], cvs, L)
        assert np.max(np.abs(xi[w].detach().cpu().numpy() - xr) / xr) <= 1e-6
        xb = k.cpu().numpy() * (xr - xi0.cpu().numpy())
        assert rel_inf(g[off[w]:off[w + 1]], np.tensordot(xb, J, axes=1)) <= 1e-5
