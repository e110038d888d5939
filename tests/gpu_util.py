"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np
import torch

from paper_2301_04835_amd import Sampler

TWO_PI = 2 * np.pi


def rel_inf(a, b):
    """max |a - b| / max |b| (inf-norm relative error)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))


def dense_jac(J_slots, atom, cv, n_atoms, D):
    """Sum sparse Jacobian slots (n_slots x 3) into a dense D x n_atoms x 3."""
    out = np.zeros((D, n_atoms, 3))
    np.add.at(out, (cv, atom), np.asarray(J_slots, dtype=np.float64))
    return out


def make_metad(cvs, sigma, height, temperature=300.0, bias_factor=None, stride=500, capacity=4096,
               atom_off=None, hill_capacity=None, box=None, tile=None, grid=0):
    s = Sampler(0)
    s.add_cvs(cvs)
    if box is not None:
        s.set_box(box)
    if atom_off is not None:
        s.set_walkers(atom_off, hill_capacity)
    s.metad(sigma, height, temperature, bias_factor, stride, capacity)
    s.bind()
    if tile is not None:
        s.set_tuning(tile, grid)
    return s


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
