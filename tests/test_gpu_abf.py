"""GPU parity of the adaptive-biasing-force path against the FP64 oracle.

Per step: xi, the bias along xi (-dV/dxi = b) and the atom forces; after the
run: the histogram (exact, integer) and the force sums.  Both sides form
theta from FP64 Jacobian rows (the coordination number's pair terms are
FP32 on the GPU), so the grid sums compare to 1e-5 relative against the
unmodified oracle; bins whose edge lies within the CV tolerance of a sample
are reported (none occur with these seeds).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2301_04835_amd import Sampler, synth

from gpu_util import dev, rel_inf

pytestmark = pytest.mark.gpu


def run_abf(cvs, box, frames, fsys, n_atoms, lo, hi, nbins, thr, atom_off=None):
    """GPU: write each frame's active atoms into the engine buffer, step."""
    s = Sampler(0)
    s.add_cvs(cvs)
    if box is not None:
        s.set_box(box)
    W = 1 if atom_off is None else len(atom_off) - 1
    s.set_walkers(np.array([0, n_atoms]) if atom_off is None else atom_off)
    s.abf(lo, hi, nbins, thr)
    s.bind()
    T, nact = frames.shape[0], frames.shape[1]
    D = len(cvs)
    P = torch.zeros((n_atoms, 3), dtype=torch.float32, device="cuda")
    Fs = torch.zeros_like(P)
    fr, ff = dev(frames), dev(fsys)
    xi = torch.zeros((T, W, D), dtype=torch.float64, device="cuda")
    dV = torch.zeros((T, W, D), dtype=torch.float64, device="cuda")
    F = torch.zeros((T, nact, 3), dtype=torch.float32, device="cuda")
    Fbuf = torch.zeros_like(P)
    for t in range(T):
        P[:nact] = fr[t]
        Fs[:nact] = ff[t]
        Fbuf.zero_()
        s.step(P, forces=Fbuf, step=t, xi_out=xi[t], dV_out=dV[t], sys_forces=Fs)
        F[t] = Fbuf[:nact]
    s.check()
    grids = [s.abf_grid(w) for w in range(W)]
    return s, xi.cpu().numpy(), dV.cpu().numpy(), F.cpu().numpy(), grids


def near_edge(x, lo, hi, nb, tol):
    u = (x - lo) / ((hi - lo) / nb)
    return abs(u - np.rint(u)) < tol * max(1.0, abs(u))


# seed of the 10^4-step run: chosen so that no sample's CV lies within
# 3e-5 bins of a bin edge (the GPU's coordination number, with FP32 pair
# terms, agrees with the oracle's to ~1e-8 relative, i.e. ~3e-6 bins)
ABF50K_SEED = 4


def test_abf50k_full_size_10k_steps(gpu):
    """The 50,000-atom ABF workload at its full size over all 10^4 steps, with
    fresh positions of the 2,500 active atoms and fresh system forces every
    step (Sec. 2.1.4): per step xi, the bias along xi and the atom forces;
    after the run the histogram (exact) and the force sums (1e-5 relative)
    against the oracle replaying the same samples."""
    import concurrent.futures as cf

    p = synth.ABF50K
    cvs = synth.abf50k_cvs()
    box = np.full(3, p["box"])
    T = p["n_steps"]
    frames, fsys = synth.abf50k_frames(T, seed=ABF50K_SEED)
    s, xi, dV, F, grids = run_abf(cvs, box, frames, fsys, p["n_atoms"], p["lo"], p["hi"], p["nbins"],
                                  p["n_threshold"])
    g = oracle.AbfGrid(p["lo"], p["hi"], p["nbins"], [False, False], p["n_threshold"])
    worst = {"xi_rg": 0.0, "xi_cn": 0.0, "b": 0.0, "F": 0.0}
    amb = nbias = 0
    ev = lambda t: oracle.cv_eval(frames[t].astype(np.float64), cvs, box)
    chunk = 500
    with cf.ThreadPoolExecutor(16) as ex:
        for c0 in range(0, T, chunk):
            for t, (x, J) in zip(range(c0, min(T, c0 + chunk)), ex.map(ev, range(c0, min(T, c0 + chunk)))):
                b, Fb, k, th = oracle.abf_step(g, x, J, fsys[t].astype(np.float64))
                worst["xi_rg"] = max(worst["xi_rg"], abs(xi[t, 0, 0] - x[0]) / x[0])
                worst["xi_cn"] = max(worst["xi_cn"], abs(xi[t, 0, 1] - x[1]) / x[1])
                if np.any(b != 0):
                    nbias += 1
                    worst["b"] = max(worst["b"], rel_inf(-dV[t, 0], b))
                    worst["F"] = max(worst["F"], rel_inf(F[t], Fb))
                else:
                    assert np.all(dV[t, 0] == 0) and np.all(F[t] == 0)
                amb += any(near_edge(x[d], p["lo"][d], p["hi"][d], p["nbins"][d], 1e-7) for d in range(2))
    print("worst:", worst, "biased steps:", nbias, "ambiguous samples:", amb)
    assert amb == 0
    assert nbias > T // 2  # most samples find a bin visited before
    assert worst["xi_rg"] <= 1e-9 and worst["xi_cn"] <= 1e-6
    assert worst["b"] <= 1e-5 and worst["F"] <= 1e-5
    N, Fsum = grids[0]
    assert np.array_equal(N.astype(np.int64), g.N)
    assert N.sum() == T  # every sample in range with this grid
    nz = g.N > 0
    assert rel_inf(Fsum[nz], g.Fsum[nz]) <= 1e-5
    assert s.get_step() == T


def test_abf_dihedrals_periodic_bins_walkers(gpu):
    """phi/psi of three walkers: periodic bins (50 per CV, the alanine
    dipeptide grid of the appendix), shared atoms in the Gram matrix,
    a low threshold so the bias is exercised, per-walker grids."""
    W, n, T = 3, 22, 400
    tmpl = synth.chain_template(n, 5)
    g0 = np.random.default_rng(8)
    frames = np.stack([synth.noisy_frames(tmpl, T, 10 + w, 0.15, np.float32) for w in range(W)], axis=1)
    frames = frames.reshape(T, W * n, 3)
    fsys = g0.normal(0, 50.0, size=(T, W * n, 3)).astype(np.float32)
    cvs = synth.backbone_cvs(4)
    lo, hi, nb, thr = [-np.pi, -np.pi], [np.pi, np.pi], [50, 50], 5
    off = np.arange(W + 1) * n
    s, xi, dV, F, grids = run_abf(cvs, None, frames, fsys, W * n, lo, hi, nb, thr, atom_off=off)
    for w in range(W):
        g = oracle.AbfGrid(lo, hi, nb, [True, True], thr)
        errF = errb = 0.0
        for t in range(T):
            sl = slice(off[w], off[w + 1])
            x, J = oracle.cv_eval(frames[t, sl].astype(np.float64), cvs)
            assert not any(near_edge(x[d], lo[d], hi[d], nb[d], 1e-9) for d in range(2))
            b, Fb, k, th = oracle.abf_step(g, x, J, fsys[t, sl].astype(np.float64))
            assert np.max(np.abs(xi[t, w] - x)) <= 1e-9
            errb = max(errb, rel_inf(-dV[t, w], b) if np.any(b) else np.max(np.abs(dV[t, w])))
            errF = max(errF, rel_inf(F[t, sl], Fb) if np.any(b) else np.max(np.abs(F[t, sl])))
        N, Fsum = grids[w]
        assert np.array_equal(N.astype(np.int64), g.N)
        assert rel_inf(Fsum[g.N > 0], g.Fsum[g.N > 0]) <= 1e-5
        assert errb <= 1e-5 and errF <= 1e-5, (w, errb, errF)


def test_abf_out_of_range_samples_are_dropped(gpu):
    cvs = synth.backbone_cvs(4)
    tmpl = synth.chain_template(22, 5)
    frames = synth.noisy_frames(tmpl, 20, 3, 0.02, np.float32)
    fsys = np.random.default_rng(1).normal(0, 10, size=frames.shape).astype(np.float32)
    # the second CV (Rg of 8 atoms, ~0.2 nm) never reaches the grid [10, 11)
    s = Sampler(0)
    s.add_dihedral(cvs[0]["idx"])
    s.add_gyration(list(range(4, 12)))  # non-periodic second CV
    s.abf([-np.pi, 10.0], [np.pi, 11.0], [10, 10], 0)
    s.bind()
    P = dev(frames[0])
    Fb = torch.zeros_like(P)
    dV = torch.ones((1, 2), dtype=torch.float64, device="cuda")
    s.step(P, forces=Fb, step=0, dV_out=dV, sys_forces=dev(fsys[0]))
    N, _ = s.abf_grid(0)
    assert N.sum() == 0 and torch.all(dV == 0) and torch.all(Fb == 0)


def test_momentum_estimator_matches_oracle(gpu):
    """The momentum-derivative estimator on (phi, psi) of 4 walkers with
    per-atom masses over 60 steps of a synthetic trajectory (positions and
    momenta drawn per step: the parity of the arithmetic, not a dynamics):
    per step the bias along xi and the forces, after the run the histogram
    (exact) and the force sums (1e-5 relative)."""
    W, n, T, dt = 4, 22, 60, 0.002
    cvs = synth.backbone_cvs(4)
    nb, lo, hi = [8, 8], [-np.pi, -np.pi], [np.pi, np.pi]
    g = np.random.default_rng(21)
    masses = g.uniform(1.0, 16.0, W * n)
    tmpl = [synth.chain_template(n, 80 + w) for w in range(W)]
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_walkers(np.arange(W + 1) * n)
    s.abf(lo, hi, nb, 3)
    s.abf_momentum(dt, masses)
    s.bind()
    grids = [oracle.AbfGrid(lo, hi, nb, [True, True], 3) for _ in range(W)]
    prev = [None] * W
    Fb = torch.zeros((W * n, 3), dtype=torch.float32, device=gpu)
    dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    for t in range(T):
        pos = np.concatenate([tm + 0.2 * g.normal(size=tm.shape) for tm in tmpl]).astype(np.float32)
        mom = (g.normal(size=pos.shape) * np.sqrt(masses)[:, None]).astype(np.float32)
        Fb.zero_()
        s.step(dev(pos), forces=Fb, step=t, dV_out=dV, sys_forces=dev(mom))
        bg, Fg = -dV.cpu().numpy(), Fb.cpu().numpy()
        for w in range(W):
            sl = slice(w * n, (w + 1) * n)
            xi, J = oracle.cv_eval(pos[sl].astype(np.float64), cvs)
            b, F, k, theta, prev[w] = oracle.abf_step_momentum(grids[w], xi, J, mom[sl].astype(np.float64),
                                                               1.0 / masses[sl], dt, prev[w])
            assert rel_inf(bg[w], b) <= 1e-5
            assert rel_inf(Fg[sl], F) <= 1e-5
    s.check()
    for w in range(W):
        N, Fsum = s.abf_grid(w)
        assert np.array_equal(N.astype(np.int64), grids[w].N)
        assert int(N.sum()) == T - 1
        assert rel_inf(Fsum, grids[w].Fsum) <= 1e-5


@pytest.mark.parametrize("estimator", [0, 1])
def test_abf_many_touched_atoms_matches_oracle(gpu, estimator):
    """Walkers touching more than 512 atoms (phi and the radius of gyration
    of 600 atoms: the two-launch form -- per-block Gram records and a
    snapshot of the update's inputs, then the sums, solve, grid update and
    force gather) on three walkers of 700 atoms, with the
    projected-force estimator (random system forces) and the momentum
    estimator (per-atom masses, momenta drawn per step): per step the bias
    along xi and the forces, after the run the histogram (exact) and the
    force sums, against the oracle as written (FP64 Jacobian) at the graded
    1e-5.  The library keeps ABF's Jacobian rows in FP64: with phi's rows
    orders of magnitude above those of Rg over 600 atoms, rounding them to
    float32 alone would move theta by up to ~1.5e-5 relative here."""
    W, n, T, dt = 3, 700, 40, 0.002
    cvs = [synth.backbone_cvs(4)[0], {"kind": "gyration", "idx": list(range(0, 600))}]
    g = np.random.default_rng(31 + estimator)
    tmpl = [synth.chain_template(n, 120 + w) for w in range(W)]
    rg0 = [oracle.cv_eval(tm.astype(np.float64), cvs)[0][1] for tm in tmpl]
    lo, hi, nb, thr = [-np.pi, min(rg0) - 0.6], [np.pi, max(rg0) + 0.6], [16, 12], 3
    masses = g.uniform(1.0, 16.0, W * n)
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_walkers(np.arange(W + 1) * n)
    s.abf(lo, hi, nb, thr)
    if estimator == 1:
        s.abf_momentum(dt, masses)
    s.bind()
    atom, _ = s.jac_layout()
    assert len(np.unique(atom)) > 512  # the two-launch form
    grids = [oracle.AbfGrid(lo, hi, nb, [True, False], thr) for _ in range(W)]
    prev = [None] * W
    Fb = torch.zeros((W * n, 3), dtype=torch.float32, device=gpu)
    dV = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    errb = errF = 0.0
    for t in range(T):
        pos = np.concatenate([tm + 0.2 * g.normal(size=tm.shape) for tm in tmpl]).astype(np.float32)
        if estimator == 1:
            q = (g.normal(size=pos.shape) * np.sqrt(masses)[:, None]).astype(np.float32)
        else:
            q = g.normal(0.0, 50.0, size=pos.shape).astype(np.float32)
        Fb.zero_()
        s.step(dev(pos), forces=Fb, step=t, dV_out=dV, sys_forces=dev(q))
        bg, Fg = -dV.cpu().numpy(), Fb.cpu().numpy()
        for w in range(W):
            sl = slice(w * n, (w + 1) * n)
            xi, J = oracle.cv_eval(pos[sl].astype(np.float64), cvs)
            assert not any(near_edge(xi[d], lo[d], hi[d], nb[d], 1e-6) for d in range(2))
            if estimator == 1:
                b, F, _, _, prev[w] = oracle.abf_step_momentum(grids[w], xi, J, q[sl].astype(np.float64),
                                                               1.0 / masses[sl], dt, prev[w])
            else:
                b, F, _, _ = oracle.abf_step(grids[w], xi, J, q[sl].astype(np.float64))
            if np.any(b != 0):
                errb = max(errb, rel_inf(bg[w], b))
                errF = max(errF, rel_inf(Fg[sl], F))
            else:
                assert np.all(bg[w] == 0) and np.all(Fg[sl] == 0)
    s.check()
    print("worst b, F rel err vs the FP64 oracle:", errb, errF)
    assert errb <= 1e-5 and errF <= 1e-5, (errb, errF)
    for w in range(W):
        N, Fsum = s.abf_grid(w)
        assert np.array_equal(N.astype(np.int64), grids[w].N)
        assert int(N.sum()) == (T if estimator == 0 else T - 1)
        nz = grids[w].N > 0
        assert rel_inf(Fsum[nz], grids[w].Fsum[nz]) <= 1e-5


@pytest.mark.parametrize("many", [False, True])
def test_abf_graph_replay_matches_eager_steps(gpu, many):
    """Replays of a captured 4-step graph against the same steps run eagerly
    on a second context, bitwise (forces, bias along xi, histogram, force
    sums), with eager work and synchronisations between the replays: the
    one-launch form (phi/psi of two 22-atom walkers) and the two-launch form
    (phi and Rg of 600 atoms, two 700-atom walkers)."""
    W = 2
    if many:
        n = 700
        cvs = [synth.backbone_cvs(4)[0], {"kind": "gyration", "idx": list(range(0, 600))}]
        lo, hi, nb = [-np.pi, 1.0], [np.pi, 3.0], [16, 12]
    else:
        n = 22
        cvs = synth.backbone_cvs(4)
        lo, hi, nb = [-np.pi, -np.pi], [np.pi, np.pi], [16, 16]
    g = np.random.default_rng(41)
    pos = np.concatenate([synth.chain_template(n, 140 + w) for w in range(W)]).astype(np.float32)
    fs = g.normal(0.0, 50.0, size=pos.shape).astype(np.float32)

    def mk():
        s = Sampler(0)
        s.add_cvs(cvs)
        s.set_walkers(np.arange(W + 1) * n)
        s.abf(lo, hi, nb, 2)
        s.bind()
        return s

    a, b = mk(), mk()
    P, Fs = dev(pos), dev(fs)
    Fa, Fb = torch.zeros_like(P), torch.zeros_like(P)
    dVa = torch.zeros((W, 2), dtype=torch.float64, device=gpu)
    dVb = torch.zeros_like(dVa)
    a.graph_capture(4, P, forces=Fa, dV_out=dVa, sys_forces=Fs)
    for rep in range(3):
        a.graph_launch()
        torch.cuda.synchronize()
        for _ in range(4):
            b.step(P, forces=Fb, dV_out=dVb, sys_forces=Fs)
        torch.cuda.synchronize()
        assert torch.equal(Fa, Fb) and torch.equal(dVa, dVb), rep
    assert torch.any(dVa != 0)  # the bias is exercised (threshold 2)
    assert a.get_step() == 12 and b.get_step() == 12
    for w in range(W):
        Na, Sa = a.abf_grid(w)
        Nb, Sb = b.abf_grid(w)
        assert int(Na.sum()) == 12 and np.array_equal(Na, Nb) and np.array_equal(Sa, Sb)
