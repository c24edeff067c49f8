"""FP64 reference of the spectral-window network (oracle).

Not in the paper: the learned spectral window predicts, from the truncated-FFT features of an
operator's coefficient field (Algorithm 2's P_low, here 3 tensor channels x 16 x 16 complex
coefficients fed as 6 real channels), the filter window [lambda_1, lambda_{L+1}] of Section 2.2
(log scale) and a filter degree.  Four layers:

    conv 3x3, 6 -> 16 channels, stride 1, zero padding 1, ReLU      (16 x 16 -> 16 x 16)
    conv 3x3, 16 -> 32 channels, stride 2, zero padding 1, ReLU     (16 x 16 -> 8 x 8)
    dense 2048 -> 64, ReLU
    dense 64 -> 3

Parameters are one flat vector in this order (row-major within each array): W1[16,6,3,3], b1[16],
W2[32,16,3,3], b2[32], W3[64,2048], b3[64], W4[3,64], b4[3].  Loss: mean over samples and outputs
of (y - t)^2 / 2.  Forward and backward are written out by hand (no autodiff) so that each
gradient can be read against the layer it belongs to.
"""
from __future__ import annotations

import numpy as np

SHAPES = [("W1", (16, 6, 3, 3)), ("b1", (16,)), ("W2", (32, 16, 3, 3)), ("b2", (32,)),
          ("W3", (64, 2048)), ("b3", (64,)), ("W4", (3, 64)), ("b4", (3,))]
COUNT = int(sum(np.prod(s) for _, s in SHAPES))


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        size = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shp)
        o += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SHAPES])


def conv2d(x, W, b, stride):
    """x [n, ci, H, W], W [co, ci, 3, 3], zero padding 1."""
    n, ci, H, Wd = x.shape
    co = W.shape[0]
    Ho, Wo = (H - 1) // stride + 1, (Wd - 1) // stride + 1
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    y = np.zeros((n, co, Ho, Wo)) + b[None, :, None, None]
    for kh in range(3):
        for kw in range(3):
            patch = xp[:, :, kh:kh + stride * (Ho - 1) + 1:stride, kw:kw + stride * (Wo - 1) + 1:stride]
            y += np.einsum("nchw,oc->nohw", patch, W[:, :, kh, kw])
    return y


def conv2d_backward(x, W, dy, stride):
    """Gradients of conv2d w.r.t. x, W, b given dy."""
    n, ci, H, Wd = x.shape
    _, co, Ho, Wo = dy.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for kh in range(3):
        for kw in range(3):
            sl = (slice(None), slice(None), slice(kh, kh + stride * (Ho - 1) + 1, stride),
                  slice(kw, kw + stride * (Wo - 1) + 1, stride))
            dW[:, :, kh, kw] = np.einsum("nohw,nchw->oc", dy, xp[sl])
            dxp[sl] += np.einsum("nohw,oc->nchw", dy, W[:, :, kh, kw])
    return dxp[:, :, 1:-1, 1:-1], dW, dy.sum(axis=(0, 2, 3))


def forward(theta, x, keep=False):
    p = unpack(theta)
    z1 = conv2d(x, p["W1"], p["b1"], 1)
    a1 = np.maximum(z1, 0.0)
    z2 = conv2d(a1, p["W2"], p["b2"], 2)
    a2 = np.maximum(z2, 0.0)
    f = a2.reshape(a2.shape[0], -1)
    z3 = f @ p["W3"].T + p["b3"]
    a3 = np.maximum(z3, 0.0)
    y = a3 @ p["W4"].T + p["b4"]
    if keep:
        return y, dict(x=x, a1=a1, a2=a2, f=f, a3=a3)
    return y


def loss_and_grad(theta, x, t):
    """(loss, gradient) of mean((y - t)^2) / 2 over all samples and outputs."""
    p = unpack(theta)
    y, c = forward(theta, x, keep=True)
    n = x.shape[0]
    d = (y - t) / (n * y.shape[1])
    loss = 0.5 * np.sum((y - t) ** 2) / (n * y.shape[1])
    g = {}
    g["W4"] = d.T @ c["a3"]
    g["b4"] = d.sum(axis=0)
    da3 = (d @ p["W4"]) * (c["a3"] > 0)
    g["W3"] = da3.T @ c["f"]
    g["b3"] = da3.sum(axis=0)
    da2 = (da3 @ p["W3"]).reshape(c["a2"].shape) * (c["a2"] > 0)
    da1, g["W2"], g["b2"] = conv2d_backward(c["a1"], p["W2"], da2, 2)
    da1 = da1 * (c["a1"] > 0)
    _, g["W1"], g["b1"] = conv2d_backward(c["x"], p["W1"], da1, 1)
    return float(loss), pack(g)


def init_params(seed=0):
    """He-normal weights, zero biases (a reference initialisation for CPU tests)."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            parts[name] = np.zeros(shp)
        else:
            fan_in = int(np.prod(shp[1:]))
            parts[name] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
    return pack(parts)


def window_features(feats):
    """Truncated-FFT features (n, C, p0, p0) complex -> network input (n, 2C, p0, p0):
    channel 2c = Re, 2c+1 = Im of channel c."""
    f = np.asarray(feats)
    n, C = f.shape[:2]
    x = np.empty((n, 2 * C) + f.shape[2:])
    x[:, 0::2] = f.real
    x[:, 1::2] = f.imag
    return x


def degree_label(lam_L, lam_L1, beta, gain=1e4, lo=8, hi=128):
    """Smallest degree m with C_m(|t(lambda_L)|) >= gain over the damped interval
    [lambda_{L+1}, beta], clamped to [lo, hi]."""
    c, e = 0.5 * (lam_L1 + beta), 0.5 * (beta - lam_L1)
    t = abs((lam_L - c) / e)
    if t <= 1.0:
        return float(hi)
    return float(min(hi, max(lo, np.ceil(np.arccosh(gain) / np.arccosh(t)))))
