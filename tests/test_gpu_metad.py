"""GPU parity of the metadynamics path against the FP64 oracle.

Tolerances (forces within 1e-5 relative of the FP64 oracle on the FP32 path):
  xi      <= 1e-9 rad (dihedrals are computed in FP64 on the GPU too)
  V       <= 1e-6 relative
  dV/dxi  <= 1e-5 relative (inf-norm over the CVs of a walker)
  forces  <= 1e-5 relative (inf-norm over the atoms of a walker)
  J       <= 1e-6 relative (float32 storage of an FP64 value)
  heights <= 1e-6 relative (float32 storage)
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2301_04835_amd import synth
from paper_2301_04835_amd.api import SxError

from gpu_util import TWO_PI, dense_jac, dev, hill_v_rel_bound, make_metad, rel_inf

pytestmark = pytest.mark.gpu

KDT = oracle.KB * (6.0 - 1.0) * 300.0  # bias factor 6, T = 300 K


# ------------------------------------------------------------------ 22 atoms
def test_wtmd22_1000_steps(gpu):
    p = synth.WTMD22
    d = synth.wtmd22_inputs()
    cvs = d["cvs"]
    C = d["centers"]
    H = oracle.wt_sequence(C.astype(np.float64), p["w"], KDT, p["sigma"], [TWO_PI, TWO_PI], round_f32=True)
    H = H.astype(np.float32)
    nsteps = d["frames"].shape[0]
    s = make_metad(cvs, p["sigma"], p["w"], p["T"], p["bias_factor"], p["stride"], capacity=2000 + 8)
    s.hills_set(0, C, H)
    frames = dev(d["frames"])
    xi = torch.zeros((nsteps, 2), dtype=torch.float64, device=gpu)
    V = torch.zeros(nsteps, dtype=torch.float64, device=gpu)
    dV = torch.zeros((nsteps, 2), dtype=torch.float64, device=gpu)
    F = torch.zeros((nsteps, 22, 3), dtype=torch.float32, device=gpu)
    Js = []
    for t in range(nsteps):
        if t % 50 == 0:
            Js.append((t, s.eval_cv(frames[t])[1].clone()))
        s.step(frames[t], forces=F[t], step=t, xi_out=xi[t], V_out=V[t], dV_out=dV[t])
    s.check()
    assert s.get_step() == nsteps
    xi, V, dV, F = (x.cpu().numpy() for x in (xi, V, dV, F))
    atom, cvi = s.jac_layout()
    Jmap = {t: dense_jac(j[0].cpu().numpy(), atom, cvi, 22, 2) for t, j in Js}
    # oracle replay
    Cr = C.astype(np.float64).tolist()
    Hr = H.astype(np.float64).tolist()
    worst = {"xi": 0, "V": 0, "dV": 0, "F": 0, "J": 0}
    for t in range(nsteps):
        o = oracle.metad_step(d["frames"][t], cvs, np.array(Cr), np.array(Hr), p["sigma"], p["w"], KDT, p["stride"], t)
        worst["xi"] = max(worst["xi"], np.max(np.abs(xi[t] - o["xi"])))
        worst["V"] = max(worst["V"], abs(V[t] - o["V"]) / abs(o["V"]))
        worst["dV"] = max(worst["dV"], rel_inf(dV[t], o["dV"]))
        worst["F"] = max(worst["F"], rel_inf(F[t], o["F"]))
        if t in Jmap:
            worst["J"] = max(worst["J"], rel_inf(Jmap[t], o["J"]))
        if o["deposit"] is not None:
            Cr.append(np.float32(o["deposit"][0]).astype(np.float64).tolist())
            Hr.append(float(np.float32(o["deposit"][1])))
    print("worst errors:", worst)
    assert worst["xi"] <= 1e-9
    assert worst["V"] <= 1e-6
    assert worst["dV"] <= 1e-5
    assert worst["F"] <= 1e-5
    assert worst["J"] <= 1e-6
    # deposits at steps 0 and 500
    c2, h2 = s.hills_get(0)
    assert c2.shape[0] == 2002
    assert np.array_equal(c2[:2000], C) and np.array_equal(h2[:2000], H)
    assert np.array_equal(c2[2000:].astype(np.float64), np.array(Cr[2000:], dtype=np.float32).astype(np.float64))
    assert rel_inf(h2[2000:], np.array(Hr[2000:])) <= 1e-6


def test_one_tile_step_matches_the_two_kernel_step(gpu):
    """A single walker whose capacity fits one tile takes the one-launch step
    (the workgroup that sums the tile also finalizes); the same walker beside
    a second one takes the tile kernel and the finalize kernel.  With a
    deposit every step over 40 steps, walker 0's xi, V, dV/dxi, forces and
    hills agree bit for bit between the two."""
    p = synth.WTMD22
    T = 40
    d = synth.wtmd22_inputs(n_steps=T)
    cvs, C = d["cvs"], d["centers"]
    H = np.full(C.shape[0], p["w"], dtype=np.float32)
    cap = C.shape[0] + 64
    one = make_metad(cvs, p["sigma"], p["w"], p["T"], p["bias_factor"], 1, capacity=cap)
    two = make_metad(cvs, p["sigma"], p["w"], p["T"], p["bias_factor"], 1, capacity=cap,
                     atom_off=np.array([0, 22, 44]), hill_capacity=[cap, cap])
    one.hills_set(0, C, H)
    two.hills_set(0, C, H)
    two.hills_set(1, C[::-1].copy(), H)
    f1 = dev(d["frames"])
    f2 = dev(np.concatenate([d["frames"], d["frames"][::-1]], axis=1))
    z = lambda *sh, dt=torch.float64: torch.zeros(sh, dtype=dt, device=gpu)
    o1 = (z(T, 22, 3, dt=torch.float32), z(T, 1, 2), z(T, 1), z(T, 1, 2))
    o2 = (z(T, 44, 3, dt=torch.float32), z(T, 2, 2), z(T, 2), z(T, 2, 2))
    for t in range(T):
        one.step(f1[t], forces=o1[0][t], step=t, xi_out=o1[1][t], V_out=o1[2][t], dV_out=o1[3][t])
        two.step(f2[t], forces=o2[0][t], step=t, xi_out=o2[1][t], V_out=o2[2][t], dV_out=o2[3][t])
    one.check()
    two.check()
    F1, x1, V1, dV1 = (x.cpu().numpy() for x in o1)
    F2, x2, V2, dV2 = (x.cpu().numpy() for x in o2)
    assert np.array_equal(F1, F2[:, :22]) and np.any(F1 != 0)
    assert np.array_equal(x1[:, 0], x2[:, 0])
    assert np.array_equal(V1[:, 0], V2[:, 0])
    assert np.array_equal(dV1[:, 0], dV2[:, 0])
    c1, h1 = one.hills_get(0)
    c2, h2 = two.hills_get(0)
    assert c1.shape[0] == C.shape[0] + T
    assert np.array_equal(c1, c2) and np.array_equal(h1, h2)


def test_sequential_deposits_follow_wt_law(gpu):
    """Heights of hills deposited one after another obey h = w exp(-V/(k dT))."""
    K = 300
    C = synth.uniform_centers(K, 2, seed=77)
    s = make_metad(synth.backbone_cvs(0), [0.35, 0.35], 1.2, 300.0, 6.0, stride=1, capacity=K + 4)
    xs = dev(C.astype(np.float64))
    for k in range(K):
        s.deposit(xs[k:k + 1])
    c, h = s.hills_get(0)
    ref = oracle.wt_sequence(C.astype(np.float64), 1.2, KDT, [0.35, 0.35], [TWO_PI] * 2, round_f32=True)
    assert np.array_equal(c, C)
    assert rel_inf(h, ref) <= 1e-6
    # plain metadynamics (no bias factor): constant height
    s2 = make_metad(synth.backbone_cvs(0), [0.35, 0.35], 1.2, 300.0, None, stride=1, capacity=16)
    for k in range(5):
        s2.deposit(xs[k:k + 1])
    assert np.all(s2.hills_get(0)[1] == np.float32(1.2))


# --------------------------------------------------------------- walkers
def _walkers(counts, caps, seed, n_atoms=30, dtype=np.float32):
    W = len(counts)
    g = np.random.default_rng(seed)
    tmpl = synth.chain_template(8, seed)
    off = np.arange(W + 1, dtype=np.int64) * n_atoms
    pos = g.uniform(-1, 1, size=(W * n_atoms, 3))
    for w in range(W):
        pos[off[w]:off[w] + 8] = tmpl + g.normal(0, 0.05, size=tmpl.shape)
    hills = [(synth.uniform_centers(k, 2, seed + 10 + w), synth.uniform_heights(k, seed + 1000 + w))
             for w, k in enumerate(counts)]
    return pos.astype(dtype), off, hills


def _oracle_walkers(pos, off, hills, cvs, sigma, W):
    out = []
    for w in range(W):
        x = pos[off[w]:off[w + 1]].astype(np.float64)
        xi, J = oracle.cv_eval(x, cvs)
        c, h = hills[w]
        if len(h):
            V, dV = oracle.hillsum(xi, c.astype(np.float64), h.astype(np.float64), sigma, [TWO_PI] * 2)
        else:
            V, dV = 0.0, np.zeros(2)
        out.append((xi, V, dV, oracle.chain_rule(-dV, J)))
    return out


@pytest.mark.parametrize("tile,grid", [(1024, 0), (2048, 3), (4096, 0), (8192, 1), (4096, 300)])
def test_ragged_walkers_all_tilings(gpu, tile, grid):
    counts = [0, 1, 3, 1023, 1024, 1025, 5000, 17]
    caps = [1, 4, 8, 1024, 1028, 2100, 5001, 40000]
    cvs = synth.backbone_cvs(1)
    sig = [0.35, 0.3]
    pos, off, hills = _walkers(counts, caps, 5)
    s = make_metad(cvs, sig, 1.2, 300.0, 6.0, 500, atom_off=off, hill_capacity=caps, tile=tile, grid=grid)
    for w, (c, h) in enumerate(hills):
        s.hills_set(w, c, h)
    W = len(counts)
    P = dev(pos)
    F = torch.zeros_like(P)
    xi = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    V = torch.zeros(W, dtype=torch.float64, device=gpu)
    dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    s.step(P, forces=F, step=3, xi_out=xi, V_out=V, dV_out=dV)
    s.check()
    ref = _oracle_walkers(pos, off, hills, cvs, sig, W)
    Fh, xh, Vh, dVh = F.cpu().numpy(), xi.cpu().numpy(), V.cpu().numpy(), dV.cpu().numpy()
    for w in range(W):
        rx, rV, rdV, rF = ref[w]
        assert np.max(np.abs(xh[w] - rx)) <= 1e-9
        if counts[w] == 0:
            assert Vh[w] == 0.0 and np.all(dVh[w] == 0.0)
            assert np.all(Fh[off[w]:off[w + 1]] == 0.0)
            continue
        assert abs(Vh[w] - rV) <= 1e-6 * abs(rV)
        assert rel_inf(dVh[w], rdV) <= 1e-5
        assert rel_inf(Fh[off[w]:off[w + 1]], rF) <= 1e-5
    # bitwise determinism (atomic-free, ordered reductions)
    F2 = torch.zeros_like(P)
    V2 = torch.zeros_like(V)
    s.step(P, forces=F2, step=3, V_out=V2)
    assert torch.equal(F, F2) and torch.equal(V, V2)


@pytest.mark.parametrize("tile,grid", [(1024, 0), (4096, 5)])
def test_growing_lists_capacity_8x_count(gpu, tile, grid):
    """Hill lists that grow during the run inside capacity reserved at 8x
    their count (Sec. 2.1.5: hills are deposited cumulatively): every step
    deposits one hill per walker (stride 1), counts start just below tile
    boundaries so live tiles appear during the run, and the tiles past the
    count leave at once.  Per step and walker: xi, V, dV/dxi and forces
    against the oracle replaying the same deposits (float32 storage); V within
    the bound its float32 terms allow (hill_v_rel_bound: 1e-6 when near
    hills dominate, more for a walker whose few hills are all far away)."""
    counts = [0, 1, 1020, 2045, 4093, 700]
    caps = [8 * max(c, 64) for c in counts]
    W, T = len(counts), 12
    cvs = synth.backbone_cvs(1)
    sig = [0.35, 0.3]
    pos0, off, hills = _walkers(counts, caps, 23)
    s = make_metad(cvs, sig, 1.2, 300.0, 6.0, 1, atom_off=off, hill_capacity=caps, tile=tile, grid=grid)
    for w, (c, h) in enumerate(hills):
        s.hills_set(w, c, h)
    g = np.random.default_rng(24)
    frames = [(pos0 + g.normal(0, 0.01, size=pos0.shape)).astype(np.float32) for _ in range(T)]
    Cr = [c.astype(np.float64).tolist() for c, _ in hills]
    Hr = [h.astype(np.float64).tolist() for _, h in hills]
    worst = {"V": 0.0, "V/bound": 0.0, "dV": 0.0, "F": 0.0}
    for t in range(T):
        P = dev(frames[t])
        F = torch.zeros_like(P)
        xi = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
        V = torch.zeros(W, dtype=torch.float64, device=gpu)
        dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
        s.step(P, forces=F, step=t, xi_out=xi, V_out=V, dV_out=dV)
        Fh, xh, Vh, dVh = F.cpu().numpy(), xi.cpu().numpy(), V.cpu().numpy(), dV.cpu().numpy()
        for w in range(W):
            o = oracle.metad_step(frames[t][off[w]:off[w + 1]], cvs, np.array(Cr[w]).reshape(-1, 2),
                                  np.array(Hr[w]), sig, 1.2, KDT, 1, t)
            assert np.max(np.abs(xh[w] - o["xi"])) <= 1e-9
            if len(Hr[w]) == 0:
                assert Vh[w] == 0.0 and np.all(dVh[w] == 0.0) and np.all(Fh[off[w]:off[w + 1]] == 0.0)
            else:
                eV = abs(Vh[w] - o["V"]) / abs(o["V"])
                bV = hill_v_rel_bound(o["xi"], Cr[w], Hr[w], sig, [TWO_PI, TWO_PI])
                worst["V"] = max(worst["V"], eV)
                worst["V/bound"] = max(worst["V/bound"], eV / bV)
                worst["dV"] = max(worst["dV"], rel_inf(dVh[w], o["dV"]))
                worst["F"] = max(worst["F"], rel_inf(Fh[off[w]:off[w + 1]], o["F"]))
            Cr[w].append(np.float32(o["deposit"][0]).astype(np.float64).tolist())
            Hr[w].append(float(np.float32(o["deposit"][1])))
    s.check()
    print("worst errors:", worst)
    assert worst["V/bound"] <= 1.0 and worst["dV"] <= 1e-5 and worst["F"] <= 1e-5
    for w in range(W):
        c, h = s.hills_get(w)
        assert c.shape[0] == counts[w] + T
        assert np.array_equal(c.astype(np.float64), np.array(Cr[w], dtype=np.float32).astype(np.float64))
        assert rel_inf(h, np.array(Hr[w])) <= 1e-6


def test_walkers_256_full_size(gpu):
    """The batched-walker workload at its full size: 256 walkers, atoms
    log-uniform in [22, 5000], 1k-50k private hills each."""
    d = synth.walkers_inputs()
    p = synth.WALKERS256
    W = p["n_walkers"]
    cvs = d["cvs"]
    caps = d["n_hills"] + 8
    s = make_metad(cvs, p["sigma"], p["w"], p["T"], p["bias_factor"], p["stride"], atom_off=d["atom_off"],
                   hill_capacity=caps)
    off, hoff = d["atom_off"], d["hill_off"]
    for w in range(W):
        s.hills_set(w, d["centers"][hoff[w]:hoff[w + 1]], d["heights"][hoff[w]:hoff[w + 1]])
    P = dev(d["pos"])
    F = torch.zeros_like(P)
    xi = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    V = torch.zeros(W, dtype=torch.float64, device=gpu)
    dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    s.step(P, forces=F, step=0, xi_out=xi, V_out=V, dV_out=dV)  # step 0: deposits
    s.check()
    # oracle: CVs per walker, batched hill sum over all walkers
    xr = np.zeros((W, 2))
    Js = []
    for w in range(W):
        xr[w], J = oracle.cv_eval(d["pos"][off[w]:off[w] + 8].astype(np.float64), cvs)
        Js.append(J)
    Vr, dVr = oracle.hillsum_batch(xr, hoff, d["centers"].astype(np.float64), d["heights"].astype(np.float64),
                                   p["sigma"], [TWO_PI] * 2, nthreads=8)
    Fh, Vh, dVh, xh = F.cpu().numpy(), V.cpu().numpy(), dV.cpu().numpy(), xi.cpu().numpy()
    assert np.max(np.abs(xh - xr)) <= 1e-9
    assert np.max(np.abs(Vh - Vr) / np.abs(Vr)) <= 1e-6
    errF = max(rel_inf(Fh[off[w]:off[w] + 8], oracle.chain_rule(-dVr[w], Js[w])) for w in range(W))
    print("max relative force error over 256 walkers:", errF)
    assert errF <= 1e-5
    assert max(rel_inf(dVh[w], dVr[w]) for w in range(W)) <= 1e-5
    assert np.all(Fh[np.concatenate([np.arange(off[w] + 8, off[w + 1]) for w in range(W)])] == 0)
    # the step-0 deposit: one hill per walker at xi with the WT height
    for w in [0, 17, 128, 255]:
        c, h = s.hills_get(w)
        assert c.shape[0] == d["n_hills"][w] + 1
        assert np.array_equal(c[-1], xr[w].astype(np.float32))
        assert abs(h[-1] - p["w"] * math.exp(-Vr[w] / KDT)) <= 1e-6 * p["w"]


def test_capacity_overflow_is_reported_and_nothing_written(gpu):
    cvs = synth.backbone_cvs(1)
    pos, off, hills = _walkers([4, 4], [4, 5], 9)
    s = make_metad(cvs, [0.35, 0.35], 1.2, 300.0, 6.0, 10, atom_off=off, hill_capacity=[4, 5])
    for w, (c, h) in enumerate(hills):
        s.hills_set(w, c, h)
    P = dev(pos)
    s.step(P, forces=torch.zeros_like(P), step=0)
    with pytest.raises(SxError) as ei:
        s.check()
    assert ei.value.status == 3
    assert s.hills_get(0)[0].shape[0] == 4      # full list untouched
    assert s.hills_get(1)[0].shape[0] == 5      # the other walker deposited
    s.check()                                    # flags were cleared


def test_graph_replay_matches_eager_steps(gpu):
    d = synth.wtmd22_inputs(n_steps=1)
    C = d["centers"][:500]
    H = synth.uniform_heights(500, 3)
    mk = lambda: make_metad(d["cvs"], [0.35, 0.35], 1.2, 300.0, 6.0, stride=2, capacity=600)
    a, b = mk(), mk()
    a.hills_set(0, C, H)
    b.hills_set(0, C, H)
    P = dev(d["frames"][0])
    Fa, Fb = torch.zeros(22, 3, dtype=torch.float32, device=gpu), torch.zeros(22, 3, dtype=torch.float32, device=gpu)
    Va, Vb = torch.zeros(1, dtype=torch.float64, device=gpu), torch.zeros(1, dtype=torch.float64, device=gpu)
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
    assert ca.shape[0] == 506 and np.array_equal(ca, cb) and np.array_equal(ha, hb)


def test_checkpoint_roundtrip_continues_bitwise(gpu):
    d = synth.wtmd22_inputs(n_steps=20)
    C = d["centers"][:300]
    H = synth.uniform_heights(300, 4)
    s = make_metad(d["cvs"], [0.35, 0.35], 1.2, 300.0, 6.0, stride=3, capacity=400)
    s.hills_set(0, C, H)
    fr = dev(d["frames"])
    F = torch.zeros((20, 22, 3), dtype=torch.float32, device=gpu)
    for t in range(10):
        s.step(fr[t], forces=F[t])
    ck = s.export_state()
    for t in range(10, 20):
        s.step(fr[t], forces=F[t])
    F1 = F.clone()
    c1 = s.hills_get(0)
    s.import_state(ck)
    assert s.get_step() == 10
    F[10:] = 0
    for t in range(10, 20):
        s.step(fr[t], forces=F[t])
    assert torch.equal(F, F1)
    c2 = s.hills_get(0)
    assert np.array_equal(c1[0], c2[0]) and np.array_equal(c1[1], c2[1])
    other = make_metad(d["cvs"], [0.35, 0.35], 1.2, 300.0, 6.0, stride=4, capacity=400)
    with pytest.raises(SxError):
        other.import_state(ck)


def test_autotune_keeps_results(gpu, tmp_path):
    d = synth.walkers_inputs(n_walkers=32, hills=(1000, 20000))
    s = make_metad(d["cvs"], [0.35, 0.35], 1.2, 300.0, 6.0, 500, atom_off=d["atom_off"],
                   hill_capacity=d["n_hills"] + 4)
    for w in range(32):
        s.hills_set(w, d["centers"][d["hill_off"][w]:d["hill_off"][w + 1]],
                    d["heights"][d["hill_off"][w]:d["hill_off"][w + 1]])
    P = dev(d["pos"])
    V0 = torch.zeros(32, dtype=torch.float64, device=gpu)
    s.step(P, forces=torch.zeros_like(P), step=1, V_out=V0)
    cache = str(tmp_path / "tune.json")
    s.autotune(P, cache)
    t, g = s.get_tuning()
    assert t in (1024, 2048, 4096, 8192)
    V1 = torch.zeros_like(V0)
    s.step(P, forces=torch.zeros_like(P), step=1, V_out=V1)
    assert torch.max(torch.abs(V1 - V0) / V0).item() <= 1e-12
    s.set_tuning(1024, 0)
    s.autotune(P, cache)  # from the cache
    assert s.get_tuning() == (t, g)


def test_invalid_arguments(gpu):
    from paper_2301_04835_amd import Sampler
    s = Sampler(0)
    with pytest.raises(SxError):
        s.add_dihedral([0, 1, 1, 2])      # repeated atom
    with pytest.raises(SxError):
        s.add_coordination([0], [1], r0=0.5, n=6, m=6)
    s.add_dihedral([0, 1, 2, 3])
    with pytest.raises(SxError):
        s.metad([-0.1], 1.0)
    with pytest.raises(SxError):
        s.metad([0.3], 1.0, 300.0, bias_factor=0.5)
    with pytest.raises(SxError) as ei:
        s.step(torch.zeros(4, 3, device=gpu))
    assert ei.value.status == 6  # not bound
