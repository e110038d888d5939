"""FP64 oracle of the bias surrogate network (test infrastructure only).

The paper's neural-network methods (ANN, Sec. 2.1.7; FUNN, Sec. 2.1.8) bias
with a small network of the CVs; the surrogate here is such a network fitted
to the metadynamics hill sum (Sec. 2.1.5):

  features  f(xi): (sin xi_d, cos xi_d) for a periodic CV d,
                   (u_d, u_d^2), u_d = (xi_d - mu_d) / s_d, otherwise
  network   z1 = W1 f + b1, a1 = tanh z1, z2 = W2 a1 + b2, a2 = tanh z2,
            y = w3 . a2 + b3                                  (V_hat)
  gradient  dy/dxi_d by the chain rule through the features

Training loss over a batch (Sobolev: value and gradient):
  L = (1/B) sum_b [ alpha (y_b - V_b)^2 + beta sum_d (dy_b/dxi_d - G_bd)^2 ]
Weight gradients follow the forward-mode tangent form of dy/dxi (one tangent
per CV through the same layers) and reverse mode over all of it; every
product is written out below in the order the derivation gives it.
Adam: Kingma & Ba (2015).

Parameters are a dict of float64 arrays: W1 (H, F), b1 (H), W2 (H, H),
b2 (H), w3 (H), b3 (1,).  ``act_round`` is an optional rounding applied to
the activation vectors that feed the H x H product (the GPU feeds them to a
BF16 matrix-core product as hi + lo pairs: ``round_bf16x2``); identity by
default.
"""
import numpy as np

PARAM_ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def n_features(periodic):
    return 2 * len(periodic)


def features(xi, periodic, mu=None, s=None):
    """f (B, F) and the feature tangents u (D, B, F) = df/dxi_d."""
    xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
    B, D = xi.shape
    f = np.zeros((B, 2 * D))
    u = np.zeros((D, B, 2 * D))
    for d in range(D):
        x = xi[:, d]
        if periodic[d]:
            f[:, 2 * d] = np.sin(x)
            f[:, 2 * d + 1] = np.cos(x)
            u[d, :, 2 * d] = np.cos(x)
            u[d, :, 2 * d + 1] = -np.sin(x)
        else:
            z = (x - mu[d]) / s[d]
            f[:, 2 * d] = z
            f[:, 2 * d + 1] = z * z
            u[d, :, 2 * d] = 1.0 / s[d]
            u[d, :, 2 * d + 1] = 2.0 * z / s[d]
    return f, u


def _ident(x):
    return x


def forward(P, xi, periodic, mu=None, s=None, act_round=_ident):
    """y (B,), dy/dxi (B, D) and the intermediates of the tangent form."""
    f, u = features(xi, periodic, mu, s)
    D = u.shape[0]
    z1 = f @ P["W1"].T + P["b1"]
    a1 = np.tanh(z1)
    a1r = act_round(a1)
    z2 = a1r @ P["W2"].T + P["b2"]
    a2 = np.tanh(z2)
    y = a2 @ P["w3"] + P["b3"][0]
    dz1 = np.stack([u[d] @ P["W1"].T for d in range(D)])          # (D, B, H)
    da1 = (1.0 - a1 * a1)[None] * dz1
    da1r = act_round(da1)
    dz2 = np.stack([da1r[d] @ P["W2"].T for d in range(D)])
    da2 = (1.0 - a2 * a2)[None] * dz2
    dy = np.stack([da2[d] @ P["w3"] for d in range(D)], axis=1)    # (B, D)
    cache = dict(f=f, u=u, z1=z1, a1=a1, a1r=a1r, a2=a2, dz1=dz1, da1=da1, da1r=da1r, dz2=dz2, da2=da2)
    return y, dy, cache


def input_grad_reverse(P, xi, periodic, mu=None, s=None):
    """dy/dxi by reverse mode (an independent route to the same gradient):
    dy/df = W1^T [(1 - a1^2) * W2^T [(1 - a2^2) * w3]]."""
    f, u = features(xi, periodic, mu, s)
    a1 = np.tanh(f @ P["W1"].T + P["b1"])
    a2 = np.tanh(a1 @ P["W2"].T + P["b2"])
    d2 = (1.0 - a2 * a2) * P["w3"]
    d1 = (d2 @ P["W2"]) * (1.0 - a1 * a1)
    dyf = d1 @ P["W1"]                                             # (B, F)
    return np.stack([np.sum(dyf * u[d], axis=1) for d in range(u.shape[0])], axis=1)


def loss_and_grads(P, xi, V, G, alpha, beta, periodic, mu=None, s=None, act_round=_ident):
    """Sobolev loss and its gradients with respect to every parameter."""
    y, dy, c = forward(P, xi, periodic, mu, s, act_round)
    B = y.shape[0]
    D = dy.shape[1]
    r0 = y - V
    r1 = dy - G
    L = (alpha * np.sum(r0 * r0) + beta * np.sum(r1 * r1)) / B
    yb = 2.0 * alpha * r0 / B                                      # dL/dy
    dyb = 2.0 * beta * r1 / B                                      # dL/d(dy_d)
    a1, a2 = c["a1"], c["a2"]
    g = {}
    # y = w3.a2 + b3, dy_d = w3.da2_d
    g["w3"] = a2.T @ yb + sum(c["da2"][d].T @ dyb[:, d] for d in range(D))
    g["b3"] = np.array([np.sum(yb)])
    da2b = np.stack([dyb[:, d:d + 1] * P["w3"][None, :] for d in range(D)])     # (D, B, H)
    # a2 feeds y and da2_d = (1 - a2^2) dz2_d
    a2b = yb[:, None] * P["w3"][None, :]
    for d in range(D):
        a2b = a2b + da2b[d] * (-2.0 * a2 * c["dz2"][d])
    dz2b = da2b * (1.0 - a2 * a2)[None]
    z2b = a2b * (1.0 - a2 * a2)
    # z2 = W2 a1r + b2, dz2_d = W2 da1r_d
    g["W2"] = z2b.T @ c["a1r"] + sum(dz2b[d].T @ c["da1r"][d] for d in range(D))
    g["b2"] = np.sum(z2b, axis=0)
    a1b = z2b @ P["W2"]
    da1b = np.stack([dz2b[d] @ P["W2"] for d in range(D)])
    for d in range(D):
        a1b = a1b + da1b[d] * (-2.0 * a1 * c["dz1"][d])
    dz1b = da1b * (1.0 - a1 * a1)[None]
    z1b = a1b * (1.0 - a1 * a1)
    # z1 = W1 f + b1, dz1_d = W1 u_d
    g["W1"] = z1b.T @ c["f"] + sum(dz1b[d].T @ c["u"][d] for d in range(D))
    g["b1"] = np.sum(z1b, axis=0)
    return L, g, y, dy


def adam_step(P, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of every parameter (t >= 1); returns new P, m, v."""
    P2, m2, v2 = {}, {}, {}
    for k in P:
        m2[k] = b1 * m[k] + (1.0 - b1) * g[k]
        v2[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mh = m2[k] / (1.0 - b1 ** t)
        vh = v2[k] / (1.0 - b2 ** t)
        P2[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P2, m2, v2


def init_params(H, F, seed):
    """Seeded uniform initialisation, +-1/sqrt(fan_in) (Glorot-like scale)."""
    g = np.random.default_rng(seed)
    return {"W1": g.uniform(-1, 1, (H, F)) / np.sqrt(F), "b1": np.zeros(H),
            "W2": g.uniform(-1, 1, (H, H)) / np.sqrt(H), "b2": np.zeros(H),
            "w3": g.uniform(-1, 1, H) / np.sqrt(H), "b3": np.zeros(1)}


def round_bf16(x):
    """Round float64 values to bfloat16 (round to nearest even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def round_bf16x2(x):
    """Value of a bfloat16 pair hi + lo with hi = bf16(x), lo = bf16(x - hi)
    (x first rounded to float32, as the GPU holds it): about 16 significant
    bits, the form in which activations enter a bf16 matrix product."""
    f = np.asarray(x, dtype=np.float32).astype(np.float64)
    hi = round_bf16(f)
    return hi + round_bf16(f - hi)
