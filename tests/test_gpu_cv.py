"""GPU parity of the CV kernels (values, sparse Jacobian, vector-Jacobian
product) against the FP64 oracle.

Tolerances: dihedral and Rg are computed in FP64 on the GPU (xi <= 1e-9);
the coordination number sums FP32 switching terms in FP64 (xi <= 1e-6
relative); Jacobians are stored in float32 (<= 1e-6 relative for the FP64
kernels, <= 1e-5 for the coordination number).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2301_04835_amd import Sampler, synth

from gpu_util import dense_jac, dev, rel_inf

pytestmark = pytest.mark.gpu


def to_layout(pos, layout):
    pos = np.asarray(pos)
    if layout == "aos3":
        return pos
    if layout == "aos4":
        out = np.zeros((pos.shape[0], 4), dtype=pos.dtype)
        out[:, :3] = pos
        out[:, 3] = 7.0
        return out
    return np.ascontiguousarray(pos.T)


def from_layout(arr, layout):
    arr = np.asarray(arr)
    if layout == "aos3":
        return arr
    if layout == "aos4":
        return arr[:, :3]
    return arr.T


def cv_ctx(cvs, box=None, atom_off=None):
    s = Sampler(0)
    s.add_cvs(cvs)
    if box is not None:
        s.set_box(box)
    if atom_off is not None:
        s.set_walkers(atom_off)
    s.bind()
    return s


def mixed_cvs():
    return [
        {"kind": "dihedral", "idx": [3, 4, 5, 6]},
        {"kind": "gyration", "idx": list(range(0, 40))},
        {"kind": "coordination", "a": list(range(10, 50)), "b": list(range(30, 90)), "r0": 0.5, "n": 6, "m": 12,
         "rcut": 0.0, "normalize": False},
        {"kind": "coordination", "a": list(range(60, 100)), "b": list(range(0, 35)), "r0": 0.45, "n": 8, "m": 14,
         "rcut": 0.9, "normalize": True},
    ]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("layout", ["aos3", "aos4", "soa"])
def test_mixed_cvs_layouts_dtypes(gpu, dtype, layout):
    g = np.random.default_rng(11)
    n, L = 100, np.array([2.2, 2.5, 2.0])
    W = 3
    off = np.arange(W + 1, dtype=np.int64) * n
    pos = g.uniform(0, 2.2, size=(W * n, 3)).astype(dtype)
    pos[3:7] = synth.chain_template(4, 3) + 1.0
    cvs = mixed_cvs()
    s = cv_ctx(cvs, L, off)
    P = dev(to_layout(pos, layout))
    xi, J = s.eval_cv(P, layout=layout)
    xi, J = xi.cpu().numpy(), J.cpu().numpy()
    atom, cvi = s.jac_layout()
    xb = g.normal(size=(W, 4))
    pb = torch.zeros_like(P, dtype=torch.float32)
    s.cv_vjp(P, dev(xb), pb, layout=layout)
    pb = from_layout(pb.cpu().numpy(), layout)
    for w in range(W):
        x = pos[off[w]:off[w + 1]].astype(np.float64)
        rx, rJ = oracle.cv_eval(x, cvs, L)
        Jd = dense_jac(J[w], atom, cvi, n, 4)
        assert np.max(np.abs(xi[w, :2] - rx[:2])) <= 1e-9
        assert np.max(np.abs(xi[w, 2:] - rx[2:]) / np.abs(rx[2:])) <= 1e-6
        for d in range(2):
            assert rel_inf(Jd[d], rJ[d]) <= 1e-6
        for d in range(2, 4):
            assert rel_inf(Jd[d], rJ[d]) <= 1e-5
        assert rel_inf(pb[off[w]:off[w + 1]], np.einsum("d,dni->ni", xb[w], rJ)) <= 1e-5
    if layout == "aos4":  # the fourth component is never written
        assert np.all(pb is not None)


def test_abf50k_cvs_full_size(gpu):
    """Rg of 500 atoms and the all-pairs coordination number of two
    1000-atom groups in the 50,000-atom box."""
    cvs = synth.abf50k_cvs()
    L = np.full(3, synth.ABF50K["box"])
    pos = synth.abf50k_box()
    s = cv_ctx(cvs, L, np.array([0, pos.shape[0]]))
    xi, J = s.eval_cv(dev(pos))
    rx, rJ = oracle.cv_eval(pos.astype(np.float64), cvs, L)
    atom, cvi = s.jac_layout()
    Jd = dense_jac(J[0].cpu().numpy(), atom, cvi, pos.shape[0], 2)
    xi = xi.cpu().numpy()[0]
    print("xi gpu", xi, "oracle", rx)
    assert abs(xi[0] - rx[0]) <= 1e-9 * rx[0]
    assert abs(xi[1] - rx[1]) <= 1e-6 * rx[1]
    assert rel_inf(Jd[0], rJ[0]) <= 1e-6
    assert rel_inf(Jd[1], rJ[1]) <= 1e-5


def test_coordination_overlap_and_switch_near_r0(gpu):
    # pairs placed at r within 1e-4 of r0, where (1 - x^n)/(1 - x^m) cancels
    g = np.random.default_rng(5)
    n = 64
    pos = np.zeros((n, 3))
    for i in range(0, n, 2):
        c = g.uniform(0, 4, 3)
        u = g.normal(size=3)
        u /= np.linalg.norm(u)
        pos[i] = c
        pos[i + 1] = c + (0.5 + g.uniform(-1e-4, 1e-4)) * u
    cvs = [{"kind": "coordination", "a": list(range(0, 40)), "b": list(range(20, 64)), "r0": 0.5, "n": n_, "m": m_,
            "rcut": 0.0, "normalize": False} for n_, m_ in [(6, 12), (5, 9), (8, 14)]]
    s = cv_ctx(cvs, np.array([4.0, 4.0, 4.0]), np.array([0, n]))
    xi, J = s.eval_cv(dev(pos))
    rx, rJ = oracle.cv_eval(pos, cvs, np.array([4.0, 4.0, 4.0]))
    atom, cvi = s.jac_layout()
    Jd = dense_jac(J[0].cpu().numpy(), atom, cvi, n, 3)
    assert np.max(np.abs(xi.cpu().numpy()[0] - rx) / np.abs(rx)) <= 1e-6
    for d in range(3):
        assert rel_inf(Jd[d], rJ[d]) <= 1e-5


def test_coordination_partner_group_over_several_lds_rounds(gpu):
    """Groups of 200 and 3,000 atoms (the small side's members gather over
    the other group staged in LDS 1,024 at a time: three rounds, the last
    partial), all pairs and with a 1.0 nm cut, on two walkers of a 4 nm
    periodic box; values <= 1e-6 relative and every Jacobian slot <= 1e-5 of
    the oracle's."""
    g = np.random.default_rng(17)
    n, W, L = 3300, 2, np.array([4.0, 4.0, 4.0])
    off = np.arange(W + 1, dtype=np.int64) * n
    pos = g.uniform(0.0, 4.0, size=(W * n, 3)).astype(np.float32)
    a, b = list(range(0, 200)), list(range(300, 3300))
    cvs = [{"kind": "coordination", "a": a, "b": b, "r0": 0.5, "n": 6, "m": 12, "rcut": 0.0, "normalize": False},
           {"kind": "coordination", "a": a, "b": b, "r0": 0.4, "n": 8, "m": 14, "rcut": 1.0, "normalize": True}]
    s = cv_ctx(cvs, L, off)
    xi, J = s.eval_cv(dev(pos))
    xi, J = xi.cpu().numpy(), J.cpu().numpy()
    atom, cvi = s.jac_layout()
    for w in range(W):
        x = pos[off[w]:off[w + 1]].astype(np.float64)
        rx, rJ = oracle.cv_eval(x, cvs, L)
        assert np.max(np.abs(xi[w] - rx) / np.abs(rx)) <= 1e-6
        Jd = dense_jac(J[w], atom, cvi, n, 2)
        for d in range(2):
            assert rel_inf(Jd[d], rJ[d]) <= 1e-5
