"""FP64 oracle of the learned search direction's U-Net (test infrastructure).

The network maps a residual to an approximate error and is appended to the
MPCG block as one more direction, so the energy minimisation of Sec. 2.2
decides its coefficient.  This module computes, in float64, what the GPU
network computes: 3x3x3 convolutions (zero padding, no bias), ReLU,
2x2x2 average pooling, nearest upsampling, channel concatenation, a final
1x1x1 convolution, a mean-squared-error loss, and the exact gradients of all
of these.  Tensors are channels-last: shape (S, S, S, C), indexed [z, y, x, c].

Storage precision: the GPU keeps weights, activations and activation
gradients in bfloat16 and accumulates in FP32.  To compare like with like,
``round_bf16`` applies the same round-to-nearest-even bfloat16 rounding where
the GPU stores a tensor (``store=True`` paths below); arithmetic stays FP64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Tuple

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(x: np.ndarray, d: Tuple[int, int, int]) -> np.ndarray:
    """out[v] = x[v + d] with zeros outside the grid."""
    out = np.zeros_like(x)
    S = x.shape[:3]
    src = []
    dst = []
    for ax in range(3):
        o = d[ax]
        n = S[ax]
        if o >= 0:
            src.append(slice(o, n))
            dst.append(slice(0, n - o))
        else:
            src.append(slice(0, n + o))
            dst.append(slice(-o, n))
    out[tuple(dst)] = x[tuple(src)]
    return out


def conv3(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """y[v, co] = sum_t sum_ci x[v + o_t, ci] w[t, co, ci]; w: (27, Cout, Cin)."""
    y = np.zeros(x.shape[:3] + (w.shape[1],))
    for t, d in enumerate(TAPS):
        y += shift(x, d) @ w[t].T
    return y


def conv3_dgrad(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv3 in x: dx[v, ci] = sum_t sum_co dy[v - o_t, co] w[t, co, ci]."""
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, d in enumerate(TAPS):
        dx += shift(dy, (-d[0], -d[1], -d[2])) @ w[t]
    return dx


def conv3_wgrad(dy: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dw[t, co, ci] = sum_v dy[v, co] x[v + o_t, ci]."""
    Cout, Cin = dy.shape[3], x.shape[3]
    dw = np.zeros((27, Cout, Cin))
    dyf = dy.reshape(-1, Cout)
    for t, d in enumerate(TAPS):
        dw[t] = dyf.T @ shift(x, d).reshape(-1, Cin)
    return dw


def conv1(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """1x1x1 convolution, w: (Cout, Cin)."""
    return x @ w.T


def avgpool2(x: np.ndarray) -> np.ndarray:
    S = x.shape[0] // 2
    return x.reshape(S, 2, S, 2, S, 2, -1).mean(axis=(1, 3, 5))


def avgpool2_bwd(dy: np.ndarray) -> np.ndarray:
    return upsample2(dy) / 8.0


def upsample2(x: np.ndarray) -> np.ndarray:
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def upsample2_bwd(dy: np.ndarray) -> np.ndarray:
    S = dy.shape[0] // 2
    return dy.reshape(S, 2, S, 2, S, 2, -1).sum(axis=(1, 3, 5))


# The U-Net: (name, kind, Cin, Cout) in order.  Channel widths 16 / 32 / 64.
LAYERS = [
    ("w1", 3, 16, 16), ("w2", 3, 16, 16),
    ("w3", 3, 16, 32), ("w4", 3, 32, 32),
    ("w5", 3, 32, 64), ("w6", 3, 64, 64),
    ("w7", 3, 96, 32), ("w8", 3, 32, 32),
    ("w9", 3, 48, 16), ("w10", 3, 16, 16),
    ("w11", 1, 16, 16),
]
IN_CHANNELS = 2     # residual and log kappa; stored padded to 16


def init_weights(seed: int) -> Dict[str, np.ndarray]:
    """He-normal initial weights (bfloat16-representable), unused input
    channels of w1 and unused output channels of w11 zero."""
    rng = np.random.default_rng(seed)
    W = {}
    for name, k, cin, cout in LAYERS:
        fan_in = (27 if k == 3 else 1) * (IN_CHANNELS if name == "w1" else cin)
        std = np.sqrt(2.0 / fan_in)
        if k == 3:
            w = rng.standard_normal((27, cout, cin)) * std
        else:
            w = rng.standard_normal((cout, cin)) * std
        if name == "w1":
            w[:, :, IN_CHANNELS:] = 0.0
        if name == "w11":
            w[1:, :] = 0.0
        W[name] = round_bf16(w)
    return W


def forward(W: Dict[str, np.ndarray], x0: np.ndarray, store: bool = True):
    """U-Net forward.  x0: (S,S,S,16) input.  Returns (output (S,S,S), cache).

    store=True rounds every stored activation to bfloat16 as the GPU does.
    """
    R = round_bf16 if store else (lambda a: a)
    c = {"x0": R(x0)}
    relu = lambda a: np.maximum(a, 0.0)
    c["e1"] = R(relu(conv3(c["x0"], W["w1"])))
    c["e2"] = R(relu(conv3(c["e1"], W["w2"])))
    c["p1"] = R(avgpool2(c["e2"]))
    c["e3"] = R(relu(conv3(c["p1"], W["w3"])))
    c["e4"] = R(relu(conv3(c["e3"], W["w4"])))
    c["p2"] = R(avgpool2(c["e4"]))
    c["b1"] = R(relu(conv3(c["p2"], W["w5"])))
    c["b2"] = R(relu(conv3(c["b1"], W["w6"])))
    c["c1"] = np.concatenate([upsample2(c["b2"]), c["e4"]], axis=3)
    c["d1"] = R(relu(conv3(c["c1"], W["w7"])))
    c["d2"] = R(relu(conv3(c["d1"], W["w8"])))
    c["c2"] = np.concatenate([upsample2(c["d2"]), c["e2"]], axis=3)
    c["d3"] = R(relu(conv3(c["c2"], W["w9"])))
    c["d4"] = R(relu(conv3(c["d3"], W["w10"])))
    out = conv1(c["d4"], W["w11"])[..., 0]
    return out, c


def backward(W: Dict[str, np.ndarray], c: dict, dout: np.ndarray, store: bool = True) -> Dict[str, np.ndarray]:
    """Gradients of sum(out * dout) with respect to every weight.

    Mirrors the GPU's sequence: every stored activation gradient is rounded
    to bfloat16 (store=True); weight gradients are exact sums (FP32 on the
    GPU).  ReLU masks use the stored post-activation (> 0).
    """
    R = round_bf16 if store else (lambda a: a)
    g = {}
    g11 = np.zeros(c["d4"].shape[:3] + (16,))
    g11[..., 0] = R(dout)
    g["w11"] = g11.reshape(-1, 16).T @ c["d4"].reshape(-1, 16)
    dd4 = R(g11 @ W["w11"])

    def relu_conv_back(name, dpost, post, inp, need_dx=True):
        dpre = dpost * (post > 0)
        g[name] = conv3_wgrad(dpre, inp)
        return R(conv3_dgrad(dpre, W[name])) if need_dx else None

    dd3 = relu_conv_back("w10", dd4, c["d4"], c["d3"])
    dc2 = relu_conv_back("w9", dd3, c["d3"], c["c2"])
    dd2 = R(upsample2_bwd(dc2[..., :32]))
    de2_skip = dc2[..., 32:]
    dd1 = relu_conv_back("w8", dd2, c["d2"], c["d1"])
    dc1 = relu_conv_back("w7", dd1, c["d1"], c["c1"])
    db2 = R(upsample2_bwd(dc1[..., :64]))
    de4_skip = dc1[..., 64:]
    db1 = relu_conv_back("w6", db2, c["b2"], c["b1"])
    dp2 = relu_conv_back("w5", db1, c["b1"], c["p2"])
    de4 = R(de4_skip + avgpool2_bwd(dp2))
    de3 = relu_conv_back("w4", de4, c["e4"], c["e3"])
    dp1 = relu_conv_back("w3", de3, c["e3"], c["p1"])
    de2 = R(de2_skip + avgpool2_bwd(dp1))
    de1 = relu_conv_back("w2", de2, c["e2"], c["e1"])
    relu_conv_back("w1", de1, c["e1"], c["x0"], need_dx=False)
    return g


def mse_loss(out: np.ndarray, target: np.ndarray, mask: np.ndarray):
    """mean over the mask of (out - target)^2 and its gradient in out."""
    n = float(mask.sum())
    diff = (out - target) * mask
    return float((diff ** 2).sum() / n), 2.0 * diff / n


def energy_loss(d: np.ndarray, r: np.ndarray, e: np.ndarray, Ad: np.ndarray):
    """Energy loss of a search direction and its gradient in d.

    For the error e with A e = r, min over c of ||e - c d||_A^2 equals
    ||e||_A^2 L with L = 1 - (d.r)^2 / ((d.A d) (e.r)) (e.r = ||e||_A^2):
    the fraction of the squared A-norm error left after the best step along
    d alone (the energy minimisation of Sec. 2.2 restricted to one
    direction).  Scale-free in d.
    dL/dd = 2 (d.r) / ((d.A d)(e.r)) ((d.r)/(d.A d) A d - r).
    All arrays are flat vectors over the n^3 nodes; Ad = A d.
    """
    a = float(d @ r)
    c = float(d @ Ad)
    E = float(e @ r)
    loss = 1.0 - a * a / (c * E)
    grad = (2.0 * a / (c * E)) * ((a / c) * Ad - r)
    return loss, grad


def marginal_energy_loss(d: np.ndarray, r: np.ndarray, e: np.ndarray, A, Z: np.ndarray, tau: float):
    """Energy loss of d on top of the block Z (columns: the level corrections
    of r), and its gradient in d.

    With Pi the A-orthogonal projection onto span(Z) (through the
    pseudo-inverse of the Gram Z^T A Z, as in the step of Sec. 2.2), the best
    combination of the columns of Z and d leaves the squared A-norm error
    ||e - Pi e||_A^2 L, L = 1 - (d.r^)^2 / ((d.A d^)(e.r^)), where r^ = A (e -
    Pi e) = r - A Z alpha (alpha = G^+ Z^T r) is the residual after the step
    over Z and A d^ = A d - A Z G^+ Z^T A d.  This is ``energy_loss`` of d
    with r and A d replaced by r^ and A d^.
    """
    from .mpcg import pinv_gram
    Q = A @ Z
    G = Z.T @ Q
    Gp = pinv_gram(0.5 * (G + G.T), tau).Gplus
    rhat = r - Q @ (Gp @ (Z.T @ r))
    Ad = A @ d
    Adhat = Ad - Q @ (Gp @ (Q.T @ d))
    return energy_loss(d, rhat, e, Adhat)


def pack_input(r: np.ndarray, logk: np.ndarray | None, n: int, S: int) -> np.ndarray:
    """Channels-last network input on the S^3 grid: channel 0 = r / rms(r),
    channel 1 = (log kappa - mean) / std (0 for Poisson); the n^3 grid sits in
    the low corner, the rest is zero."""
    x = np.zeros((S, S, S, 16))
    rr = r.reshape(n, n, n)
    rms = np.sqrt(np.mean(rr ** 2))
    x[:n, :n, :n, 0] = rr / (rms if rms > 0 else 1.0)
    if logk is not None:
        lk = logk.reshape(n, n, n)
        sd = lk.std()
        x[:n, :n, :n, 1] = (lk - lk.mean()) / (sd if sd > 0 else 1.0)
    return x
