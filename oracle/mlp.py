"""FP64 oracle of the learned importance-sampling proposal.

TEST INFRASTRUCTURE ONLY (see oracle.py): plain numpy in float64.

The proposal is a mixture of K products of logistic-normal densities over the
five unit-cube variables u of the CM-angle parameterisation (p2 in the box,
cos theta*, phi*), conditioned on the work item through an MLP:

    x (8 inputs) -> Linear 8x128 -> SiLU -> Linear 128x128 -> SiLU
                 -> Linear 128 x K(1 + 5 + 5)  = head
    head[:, 0:K]        mixture logits a_k
    head[:, K:6K]       locations mu_kd (k-major)
    head[:, 6K:11K]     log scales l_kd, clamped to [LS_MIN, LS_MAX]

With y = logit(u):
    log q_mix(y) = logsumexp_k [ log softmax(a)_k
                                 + sum_d ( -z_kd^2/2 - l_kd - log(2 pi)/2 ) ],
    z_kd = (y_d - mu_kd) exp(-l_kd).
The density on the unit cube adds the Jacobian -sum_d log(u_d (1 - u_d)),
which does not depend on the parameters.

Training loss over recorded samples (x_i, y_i, w_i = |integrand|):
    L = - sum_i w_i log q_mix(y_i | x_i) / sum_i w_i,
the cross entropy to the target density proportional to |integrand|.
Optimiser: Adam (Kingma & Ba, 2015) on FP32 master weights.
"""
from __future__ import annotations

import numpy as np

N_IN, HID, K, D = 8, 128, 8, 5
N_OUT = K * (1 + 2 * D)
LS_MIN, LS_MAX = -7.0, 3.0
LOG2PI = np.log(2.0 * np.pi)
PARAM_SHAPES = (("W1", (N_IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
                ("W3", (HID, N_OUT)), ("b3", (N_OUT,)))


def n_params() -> int:
    return sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def unflatten(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shape in PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in PARAM_SHAPES])


def bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p: dict, X, quantize=None):
    """Head outputs and the intermediates needed by the backward pass.

    quantize: optional function applied to every GEMM operand (e.g. bf16), to
    model the precision of the operands the GPU multiplies."""
    q = quantize or (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    Z1 = q(X) @ q(p["W1"]) + p["b1"]
    H1 = silu(Z1)
    Z2 = q(H1) @ q(p["W2"]) + p["b2"]
    H2 = silu(Z2)
    Y = q(H2) @ q(p["W3"]) + p["b3"]
    return Y, dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2)


def split_head(Y):
    Y = np.asarray(Y, dtype=np.float64)
    a = Y[:, :K]
    mu = Y[:, K:K + K * D].reshape(-1, K, D)
    l_raw = Y[:, K + K * D:].reshape(-1, K, D)
    return a, mu, l_raw


def log_mixture(Y, y):
    """log q_mix(y) per row (without the unit-cube Jacobian), and the pieces."""
    a, mu, l_raw = split_head(Y)
    ls = np.clip(l_raw, LS_MIN, LS_MAX)
    logpi = a - a.max(axis=1, keepdims=True)
    logpi = logpi - np.log(np.exp(logpi).sum(axis=1, keepdims=True))
    z = (np.asarray(y, dtype=np.float64)[:, None, :] - mu) * np.exp(-ls)
    lk = logpi + np.sum(-0.5 * z * z - ls - 0.5 * LOG2PI, axis=2)
    m = lk.max(axis=1, keepdims=True)
    L = (m + np.log(np.exp(lk - m).sum(axis=1, keepdims=True)))[:, 0]
    r = np.exp(lk - L[:, None])                        # responsibilities
    return L, dict(logpi=logpi, z=z, ls=ls, l_raw=l_raw, r=r)


def log_density_unit_cube(Y, u):
    """log of the mixture density on the unit cube at u (without the defensive part)."""
    u = np.asarray(u, dtype=np.float64)
    y = np.log(u) - np.log1p(-u)
    L, _ = log_mixture(Y, y)
    return L - np.sum(np.log(u) + np.log1p(-u), axis=1)


def loss_and_dY(Y, y, w):
    """Weighted NLL and its gradient with respect to the head outputs."""
    w = np.asarray(w, dtype=np.float64)
    W = w.sum()
    L, c = log_mixture(Y, y)
    loss = -np.dot(w, L) / W
    s = (w / W)[:, None]
    pi = np.exp(c["logpi"])
    da = -s * (c["r"] - pi)
    r3 = c["r"][:, :, None]
    inv = np.exp(-c["ls"])
    dmu = -s[:, :, None] * r3 * c["z"] * inv
    dls = -s[:, :, None] * r3 * (c["z"] ** 2 - 1.0)
    inside = (c["l_raw"] >= LS_MIN) & (c["l_raw"] <= LS_MAX)
    dls = np.where(inside, dls, 0.0)
    dY = np.concatenate([da, dmu.reshape(len(Y), -1), dls.reshape(len(Y), -1)], axis=1)
    return loss, dY


def backward(p: dict, cache: dict, dY, quantize=None) -> dict:
    q = quantize or (lambda a: np.asarray(a, dtype=np.float64))
    g = {}
    g["W3"] = q(cache["H2"]).T @ q(dY)
    g["b3"] = dY.sum(axis=0)
    dH2 = q(dY) @ q(p["W3"]).T
    dZ2 = dH2 * dsilu(cache["Z2"])
    g["W2"] = q(cache["H1"]).T @ q(dZ2)
    g["b2"] = dZ2.sum(axis=0)
    dH1 = q(dZ2) @ q(p["W2"]).T
    dZ1 = dH1 * dsilu(cache["Z1"])
    g["W1"] = q(cache["X"]).T @ q(dZ1)
    g["b1"] = dZ1.sum(axis=0)
    return g


def loss_and_grad(p: dict, X, y, w, quantize=None):
    Y, cache = forward(p, X, quantize)
    loss, dY = loss_and_dY(Y, y, w)
    return loss, backward(p, cache, dY, quantize)


def adam(p: dict, g: dict, state: dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8) -> dict:
    """One Adam step (bias-corrected), returns the new parameters."""
    t = state.get("t", 0) + 1
    state["t"] = t
    out = {}
    for name, _ in PARAM_SHAPES:
        m = state.setdefault("m_" + name, np.zeros_like(p[name]))
        v = state.setdefault("v_" + name, np.zeros_like(p[name]))
        m[...] = b1 * m + (1 - b1) * g[name]
        v[...] = b2 * v + (1 - b2) * g[name] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        out[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)
    return out


def table_from_head(Y, alpha: float = 0.1):
    """Proposal table (thr u32 [B,K], mu f32 [B,K,5], sigma f32 [B,K,5]).

    thr[:, 0] = floor(alpha 2^32); thr[:, k] = floor(2^32 (alpha + (1 - alpha)
    sum_{j<k} pi_j)) for k >= 1, with pi = softmax(logits)."""
    a, mu, l_raw = split_head(Y)
    pi = np.exp(a - a.max(axis=1, keepdims=True))
    pi /= pi.sum(axis=1, keepdims=True)
    cum = np.concatenate([np.zeros((len(Y), 1)), np.cumsum(pi, axis=1)[:, :-1]], axis=1)
    lo = alpha + (1.0 - alpha) * cum
    thr = np.minimum(np.floor(lo * 4294967296.0), 4294967295.0).astype(np.uint32)
    sigma = np.exp(np.clip(l_raw, LS_MIN, LS_MAX))
    return thr, mu.astype(np.float32), sigma.astype(np.float32)


def features(p1, mass_obs2, mg2, species, chan_ordinal, n_channels, p_half):
    """The eight conditioning inputs of a work item (observed node p1, its
    species' thermal mass squared, the regulator m_g^2, species index, channel
    ordinal), scaled to O(1)."""
    p_half = np.asarray(p_half, dtype=np.float64)
    pn = np.sqrt(np.sum(p_half ** 2))
    p1 = np.atleast_2d(np.asarray(p1, dtype=np.float64))
    a = np.sqrt(np.sum(p1 ** 2, axis=1))
    E1 = np.sqrt(a * a + mass_obs2)
    ch = (2.0 * chan_ordinal / (n_channels - 1) - 1.0) if n_channels > 1 else np.zeros_like(a)
    cols = [p1[:, 0] / p_half[0], p1[:, 1] / p_half[1], p1[:, 2] / p_half[2], a / pn, E1 / pn,
            np.broadcast_to(mg2 / pn ** 2, a.shape), np.broadcast_to(species / 3.0 - 1.0, a.shape),
            np.broadcast_to(ch, a.shape)]
    return np.stack(cols, axis=1)
