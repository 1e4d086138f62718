"""Plaintext integer references (test infrastructure only).

Convolution here is the CNN cross-correlation; the weight gradient is the
correlation of the padded input with the output gradient (Section 2, "Neural
Network Training"); all sums are exact int64 and results are finally taken
mod t into [0, t).
"""
import numpy as np


def conv2d_strided(x, w, P, stride):
    """y[m, y, z] = sum over c, a, b of xpad[c, y*stride + a, z*stride + b] * w[m, c, a, b]."""
    C, H, W = x.shape
    M, _, h, _ = w.shape
    xp = np.zeros((C, H + 2 * P, W + 2 * P), dtype=np.int64)
    xp[:, P:P + H, P:P + W] = x
    Ho, Wo = (H + 2 * P - h) // stride + 1, (W + 2 * P - h) // stride + 1
    y = np.zeros((M, Ho, Wo), dtype=np.int64)
    for yy in range(Ho):
        for zz in range(Wo):
            patch = xp[:, yy * stride:yy * stride + h, zz * stride:zz * stride + h]
            y[:, yy, zz] = np.einsum("mcab,cab->m", w.astype(np.int64), patch)
    return y


def conv2d(x, w, P):
    """x[C, H, W], w[M, C, h, h], stride 1, zero padding P -> y[M, Ho, Wo] (int64)."""
    C, H, W = x.shape
    M, _, h, _ = w.shape
    xp = np.zeros((C, H + 2 * P, W + 2 * P), dtype=np.int64)
    xp[:, P:P + H, P:P + W] = x
    Ho, Wo = H + 2 * P - h + 1, W + 2 * P - h + 1
    y = np.zeros((M, Ho, Wo), dtype=np.int64)
    for a in range(h):
        for b in range(h):
            patch = xp[:, a:a + Ho, b:b + Wo]            # [C, Ho, Wo]
            y += np.einsum("mc,chw->mhw", w[:, :, a, b].astype(np.int64), patch)
    return y


def conv2d_weight_grad(x, dy, P, h):
    """dW[m, c, a, b] = sum_{y,z} dy[m, y, z] * xpad[c, y+a, z+b]; x[C,H,W], dy[M,Ho,Wo]."""
    C, H, W = x.shape
    M, Ho, Wo = dy.shape
    xp = np.zeros((C, H + 2 * P, W + 2 * P), dtype=np.int64)
    xp[:, P:P + H, P:P + W] = x
    dw = np.zeros((M, C, h, h), dtype=np.int64)
    for a in range(h):
        for b in range(h):
            patch = xp[:, a:a + Ho, b:b + Wo]
            dw[:, :, a, b] = np.einsum("myz,cyz->mc", dy.astype(np.int64), patch)
    return dw


def conv2d_input_grad(dy, w, P, H, W):
    """Input gradient of conv2d (Section 2, training): dX[c, y, z] = sum over m, a, b
    of dy[m, y + P - a, z + P - b] * w[m, c, a, b] where that dy index lies in the
    output map; dy[M, Ho, Wo], w[M, C, h, h] -> dX[C, H, W] (stride 1)."""
    M, Ho, Wo = dy.shape
    _, C, h, _ = w.shape
    dx = np.zeros((C, H, W), dtype=np.int64)
    for a in range(h):
        for b in range(h):
            for y in range(H):
                yy = y + P - a
                if not 0 <= yy < Ho:
                    continue
                for z in range(W):
                    zz = z + P - b
                    if 0 <= zz < Wo:
                        dx[:, y, z] += w[:, :, a, b].astype(np.int64).T @ dy[:, yy, zz].astype(np.int64)
    return dx


def matvec(Wm, x):
    return Wm.astype(np.int64) @ x.astype(np.int64)


def mod_t(v, t):
    return np.remainder(np.asarray(v, dtype=np.int64), t)
