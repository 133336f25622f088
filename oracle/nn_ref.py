"""FP64 reference of the learned-initial-guess network (TEST INFRASTRUCTURE ONLY).

Same architecture and parameter layout as the device network: conv 3x3 s1 p1 (2->64), ReLU,
conv 3x3 s2 p1 (64->64), ReLU, per-channel mean over the 16x16 pixels added back (global
context), transposed conv 4x4 s4 (64->64), ReLU, transposed conv 2x2 s1 (64->1); flat parameters [W0 b0 W1 b1 W2 b2 W3 b3], W0/W1 as [co][ci][ky][kx], W2/W3 as
[ci][co][ky][kx].  With `bf16=True` the inputs, the weights and every stored activation are
rounded to BF16 (round to nearest even) exactly where the device rounds them; all arithmetic is
FP64.  Written with plain array slicing and sums so each layer can be read against its
definition; pinned by torch's CPU convolutions and by central finite differences.
"""
from __future__ import annotations

import numpy as np

C = 64
SHAPES = [("W0", (C, 2, 3, 3)), ("b0", (C,)), ("W1", (C, C, 3, 3)), ("b1", (C,)), ("W2", (C, C, 4, 4)),
          ("b2", (C,)), ("W3", (C, 1, 2, 2)), ("b3", (1,))]
NPARAM = int(sum(np.prod(s) for _, s in SHAPES))


def unpack(p):
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(x):
    """Round FP32 values to BF16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u >> 16) & 1) + 0x7FFF
    u = ((u + r) >> 16) << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def _conv(x, W, stride):
    """Cross-correlation with zero padding 1: out[b,o,y,x] = sum_{c,ky,kx} W[o,c,ky,kx] in[b,c,sy+ky-1,sx+kx-1]."""
    B, Ci, H, _ = x.shape
    Ho = (H + 2 - 3) // stride + 1
    xp = np.zeros((B, Ci, H + 2, H + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((B, W.shape[0], Ho, Ho))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Ho - 1) + 1:stride]
            out += np.einsum("bchw,oc->bohw", patch, W[:, :, ky, kx])
    return out


def _conv_back(dout, x, W, stride):
    """Gradients of _conv w.r.t. its input and weights."""
    B, Ci, H, _ = x.shape
    Ho = dout.shape[2]
    xp = np.zeros((B, Ci, H + 2, H + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Ho - 1) + 1, stride))
            dW[:, :, ky, kx] = np.einsum("bohw,bchw->oc", dout, xp[sl])
            dxp[sl] += np.einsum("bohw,oc->bchw", dout, W[:, :, ky, kx])
    return dxp[:, :, 1:-1, 1:-1], dW


def _convT(x, W, k, stride, Hout):
    """Transposed convolution: out[b,o,s*iy+ky,s*ix+kx] += W[c,o,ky,kx] in[b,c,iy,ix]."""
    B, Ci, H, _ = x.shape
    out = np.zeros((B, W.shape[1], Hout, Hout))
    for ky in range(k):
        for kx in range(k):
            out[:, :, ky:ky + stride * (H - 1) + 1:stride, kx:kx + stride * (H - 1) + 1:stride] += \
                np.einsum("bchw,co->bohw", x, W[:, :, ky, kx])
    return out


def _convT_back(dout, x, W, k, stride):
    B, Ci, H, _ = x.shape
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for ky in range(k):
        for kx in range(k):
            d = dout[:, :, ky:ky + stride * (H - 1) + 1:stride, kx:kx + stride * (H - 1) + 1:stride]
            dW[:, :, ky, kx] = np.einsum("bohw,bchw->co", d, x)
            dx += np.einsum("bohw,co->bchw", d, W[:, :, ky, kx])
    return dx, dW


def forward(p, x, bf=True):
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(p)
    W0, W1, W2, W3 = (r(P[k]) for k in ("W0", "W1", "W2", "W3"))
    x = r(np.asarray(x, dtype=np.float64).reshape(-1, 2, 32, 32))
    z1 = _conv(x, W0, 1) + P["b0"][None, :, None, None]
    a1 = r(np.maximum(z1, 0.0))
    z2 = _conv(a1, W1, 2) + P["b1"][None, :, None, None]
    a2 = r(np.maximum(z2, 0.0))
    a2g = r(a2 + a2.mean(axis=(2, 3), keepdims=True))      # global context
    z3 = _convT(a2g, W2, 4, 4, 64) + P["b2"][None, :, None, None]
    a3 = r(np.maximum(z3, 0.0))
    y = _convT(a3, W3, 2, 1, 65)[:, 0] + P["b3"][0]
    cache = dict(x=x, a1=a1, a2=a2, a2g=a2g, a3=a3, W0=W0, W1=W1, W2=W2, W3=W3)
    return y.reshape(y.shape[0], -1), cache


def laplacian(e):
    """5-point Laplacian 4e_ij - e_(i+-1)j - e_i(j+-1) on [B,65,65] with zero outside."""
    p = np.pad(e, ((0, 0), (1, 1), (1, 1)))
    return 4 * e - p[:, :-2, 1:-1] - p[:, 2:, 1:-1] - p[:, 1:-1, :-2] - p[:, 1:-1, 2:]


def loss_and_grad(p, x, t, bf=True, lap_weight=0.0):
    """Loss mean((y-t)^2) + w mean((L(y-t))^2) and its gradient (flat parameter layout)."""
    y, c = forward(p, x, bf)
    t = np.asarray(t, dtype=np.float64).reshape(y.shape)
    n = y.size
    e = (y - t).reshape(-1, 65, 65)
    l = laplacian(e)
    loss = float((np.sum(e ** 2) + lap_weight * np.sum(l ** 2)) / n)
    dy = ((2.0 * e + lap_weight * 2.0 * laplacian(l)) / n).reshape(-1, 1, 65, 65)
    g = {}
    g["b3"] = np.array([dy.sum()])
    da3, g["W3"] = _convT_back(dy, c["a3"], c["W3"], 2, 1)
    dz3 = da3 * (c["a3"] > 0)
    g["b2"] = dz3.sum(axis=(0, 2, 3))
    dg, g["W2"] = _convT_back(dz3, c["a2g"], c["W2"], 4, 4)
    da2 = dg + dg.mean(axis=(2, 3), keepdims=True)
    dz2 = da2 * (c["a2"] > 0)
    g["b1"] = dz2.sum(axis=(0, 2, 3))
    da1, g["W1"] = _conv_back(dz2, c["a1"], c["W1"], 2)
    dz1 = da1 * (c["a1"] > 0)
    g["b0"] = dz1.sum(axis=(0, 2, 3))
    _, g["W0"] = _conv_back(dz1, c["x"], c["W0"], 1)
    return loss, pack(g)
