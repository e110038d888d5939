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


def hill_v_rel_bound(xi, C, H, sigma, period, base=1e-6):
    """Relative error bound of a float32 hill sum V = sum_k h_k g_k at xi.
    The kernel rounds each wrapped displacement to float32 (relative u =
    2^-24) and forms the exponent in float32, so a term with exponent
    q_k = sum_d D_kd^2 / (2 sigma_d^2) carries a relative error of about
    6 u q_k, i.e. 3 u sum_d D_kd^2 / sigma_d^2; V's terms are all positive,
    so V's relative error is their e-weighted mean, plus `base` for the
    exponential, the products and the sums.  Near hills dominate V in a
    converged bias and this stays ~1e-7; a walker whose only hills are far
    away (D ~ pi at sigma 0.3) sees a few 1e-6."""
    xi = np.asarray(xi, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64).reshape(-1, len(xi))
    H = np.asarray(H, dtype=np.float64)
    if len(H) == 0:
        return base
    dl = xi[None, :] - C
    for d, p in enumerate(period):
        if p > 0:
            dl[:, d] -= p * np.rint(dl[:, d] / p)
    r = np.sum(dl ** 2 / np.asarray(sigma, dtype=np.float64) ** 2, axis=1)
    e = H * np.exp(-0.5 * r)
    V = np.sum(e)
    return base + (3.0 * 2.0 ** -24 * np.sum(e * r) / V if V > 0 else 0.0)


def hill_grad_bound(xi, C, H, sigma, period, hess, xi_tol, rel=1e-5):
    """Per-CV bound on |dV/dxi_gpu - dV/dxi_ref| for a hill sum whose
    gradient cancels: rel times the larger of max |dV/dxi| and the term scale
    S_d = sum_k h_k g_k |D_kd| / sigma_d^2 (a sum whose terms cancel carries
    a rounding error relative to the sum of their magnitudes, not to the
    result), plus what the CV tolerance xi_tol (per CV) moves the gradient
    through the bias's Hessian `hess` (D x D)."""
    xi = np.asarray(xi, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64).reshape(-1, len(xi))
    H = np.asarray(H, dtype=np.float64)
    sig2 = np.asarray(sigma, dtype=np.float64) ** 2
    dl = xi[None, :] - C
    for d, p in enumerate(period):
        if p > 0:
            dl[:, d] -= p * np.rint(dl[:, d] / p)
    e = H * np.exp(-0.5 * np.sum(dl ** 2 / sig2, axis=1))
    S = np.sum(e[:, None] * np.abs(dl), axis=0) / sig2
    g = -np.sum(e[:, None] * dl, axis=0) / sig2
    return rel * np.maximum(np.max(np.abs(g)), S) + np.abs(np.asarray(hess)) @ np.asarray(xi_tol, dtype=np.float64)


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
