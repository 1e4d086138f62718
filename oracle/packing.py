"""Correlation-aware polynomial packing (Section 3.3) and its extensions.

Test infrastructure only.  Everything is index arithmetic on integer arrays.

Single channel (Eq. 1 and Eq. 2 of Section 3.3):
    x_hat[i*O + j]               = x[i, j]
    w_hat[(h-1-i)*O + (h-1-j)]   = w[i, j]        with O = max(W, H) + h - 1.
Coefficient u*O + v of x_hat * w_hat is the full 2-D correlation
    F[u, v] = sum_{a,b} x[u-(h-1)+a, v-(h-1)+b] * w[a, b],
and a stride-1 convolution with zero padding P reads out[y, z] = F[y+h-1-P, z+h-1-P].
The product's highest degree is span = (H+h-2)*O + (W+h-2), so a single
channel fits one ring element when span + 1 <= N (the exact no-wrap condition;
the condition printed in Section 3.3 is garbled, this is the reading used).

Readings for what the paper leaves unstated:
  * channels: input channel c sits at offset c*S (S = span + 1); kernel channel
    c sits at offset -c*S, i.e. coefficient N - c*S + p carries -w (X^N = -1).
    Cross-channel terms then land in [S, N), so block 0 holds the channel sum
    when C_w = floor(N / S) channels share one polynomial; C is split into
    cb = ceil(C / C_w) blocks whose products are accumulated.
  * weight gradient (Section 2: dW is the correlation of x with dY): X is
    packed like a conv input with an h' = H_out "kernel" dY packed by Eq. 2;
    dW[m, c, a, b] is coefficient c*S + (a-P+h'-1)*O + (b-P+h'-1).
  * fully connected: x_hat[j] = x[j], w_hat[i*n_iw + n_iw-1-j] = W[i, j];
    y[i] is coefficient i*n_iw + n_iw - 1; fit (n_ow+1)*n_iw - 1 <= N.
"""
import math

import numpy as np


class ConvGeometry:
    """Geometry of a correlation-aware conv (or weight-gradient) packing."""

    def __init__(self, C, H, W, h, P, N):
        self.C, self.H, self.W, self.h, self.P, self.N = C, H, W, h, P, N
        self.O = max(W, H) + h - 1
        self.span = (H + h - 2) * self.O + (W + h - 2)
        self.S = self.span + 1
        if self.S > N:
            raise ValueError("single channel does not fit one polynomial (span+1 > N)")
        self.Cw = N // self.S
        self.cb = -(-C // self.Cw)
        self.Hout = H + 2 * P - h + 1
        self.Wout = W + 2 * P - h + 1

    def as_dict(self):
        return dict(O=self.O, span=self.span, S=self.S, Cw=self.Cw, cb=self.cb, Hout=self.Hout, Wout=self.Wout)


def pi_x(x, O, N):
    """Eq. 1 for one channel: x[H, W] -> polynomial of length N."""
    H, W = x.shape
    p = np.zeros(N, dtype=np.int64)
    for i in range(H):
        for j in range(W):
            p[i * O + j] = x[i, j]
    return p


def pi_w(w, O, N):
    """Eq. 2 for one channel: w[h, h] -> polynomial of length N."""
    h = w.shape[0]
    p = np.zeros(N, dtype=np.int64)
    for i in range(h):
        for j in range(w.shape[1]):
            p[(h - 1 - i) * O + (h - 1 - j)] = w[i, j]
    return p


def pack_conv_input(x, g):
    """x[C, H, W] -> [cb, N] integer polynomials (channel c of block k at offset (c - k*Cw)*S)."""
    out = np.zeros((g.cb, g.N), dtype=np.int64)
    for c in range(g.C):
        k, cc = divmod(c, g.Cw)
        out[k, cc * g.S:cc * g.S + g.S] += pi_x(x[c], g.O, g.N)[:g.S]
    return out


def pack_conv_weight(w, g):
    """w[M, C, h, h] -> [M, cb, N]: channel cc of a block at offset -cc*S (negated, wrapped)."""
    M = w.shape[0]
    out = np.zeros((M, g.cb, g.N), dtype=np.int64)
    for m in range(M):
        for c in range(g.C):
            k, cc = divmod(c, g.Cw)
            pw = pi_w(w[m, c], g.O, g.N)
            if cc == 0:
                out[m, k] += pw
            else:
                base = g.N - cc * g.S
                nz = np.nonzero(pw)[0]
                for e in nz:
                    out[m, k, base + e] -= pw[e]
    return out


def conv_extract(poly, g):
    """Block-0 coefficients of a decrypted product -> out[Hout, Wout]."""
    out = np.zeros((g.Hout, g.Wout), dtype=np.int64)
    for y in range(g.Hout):
        for z in range(g.Wout):
            out[y, z] = poly[(y + g.h - 1 - g.P) * g.O + (z + g.h - 1 - g.P)]
    return out


def conv_terms(B, M, cb):
    """Term lists for a batched conv: output (b, m) = sum_k ct[b, k] (x) pt[m, k]."""
    row, cti, pti = [0], [], []
    for b in range(B):
        for m in range(M):
            for k in range(cb):
                cti.append(b * cb + k)
                pti.append(m * cb + k)
            row.append(len(cti))
    return np.array(row, np.int32), np.array(cti, np.int32), np.array(pti, np.int32)


def dw_geometry(C, H, W, Hk, P, N):
    """Weight-gradient packing: X[c] (H x W) against an Hk x Hk 'kernel' dY."""
    return ConvGeometry(C, H, W, Hk, P, N)


def dw_terms(B, M, cb):
    """Term lists of the CryptoTrain-P weight-gradient update (Section 3.2):
        out[m, k] = sum_b [X_b,k] (x) (dY_b,m - r) + [dY_b,m] (x) (X_b,k - r).
    ct layout [B][cb + M] (X blocks, then dY per output channel);
    pt layout [B][M + cb] (dY - r per output channel, then X - r blocks);
    output layout [M][cb]."""
    row, cti, pti = [0], [], []
    for m in range(M):
        for k in range(cb):
            for b in range(B):
                cti.append(b * (cb + M) + k)
                pti.append(b * (M + cb) + m)
                cti.append(b * (cb + M) + cb + m)
                pti.append(b * (M + cb) + M + k)
            row.append(len(cti))
    return np.array(row, np.int32), np.array(cti, np.int32), np.array(pti, np.int32)


def dw_extract(polys, g):
    """Weight gradient from the products of a weight-gradient layer: polys[M, cb, N]
    (output (m, k) of dw_terms) -> dW[M, C, hk, hk] with hk = H + 2P - h' + 1, where
    h' = g.h is the side of the dY "kernel".  Channel c of block k = c // Cw sits at
    offset (c % Cw) * S, and dW[m, c, a, b] is the correlation coefficient at
    (a - P + h' - 1, b - P + h' - 1) of that channel (Section 2: dW is the
    correlation of the padded input with dY)."""
    M = polys.shape[0]
    hp = g.h
    hk = g.H + 2 * g.P - hp + 1
    out = np.zeros((M, g.C, hk, hk), dtype=np.int64)
    for m in range(M):
        for c in range(g.C):
            k, cc = divmod(c, g.Cw)
            for a in range(hk):
                for b in range(hk):
                    out[m, c, a, b] = polys[m, k, cc * g.S + (a - g.P + hp - 1) * g.O + (b - g.P + hp - 1)]
    return out


class FcGeometry:
    """Mat-vec packing: minimise (#CPMul, #input ct, #output ct) over the input chunk
    width n_iw (scanned upward), with n_ow = min(n_out, floor((N+1)/n_iw) - 1)."""

    def __init__(self, n_in, n_out, N):
        self.n_in, self.n_out, self.N = n_in, n_out, N
        best = None
        for n_iw in range(1, min(n_in, N) + 1):
            n_ow = min(n_out, (N + 1) // n_iw - 1)
            if n_ow < 1:
                break
            in_ct = -(-n_in // n_iw)
            out_ct = -(-n_out // n_ow)
            key = (in_ct * out_ct, in_ct, out_ct)
            if best is None or key < best[0]:
                best = (key, n_iw, n_ow)
        (self.n_cpmul, self.in_ct, self.out_ct), self.n_iw, self.n_ow = best

    def as_dict(self):
        return dict(n_iw=self.n_iw, n_ow=self.n_ow, in_ct=self.in_ct, out_ct=self.out_ct, n_cpmul=self.n_cpmul)


def pack_fc_input(x, g):
    out = np.zeros((g.in_ct, g.N), dtype=np.int64)
    for j in range(g.n_in):
        k, jj = divmod(j, g.n_iw)
        out[k, jj] = x[j]
    return out


def pack_fc_weight(Wm, g):
    """W[n_out, n_in] -> [out_ct, in_ct, N]."""
    out = np.zeros((g.out_ct, g.in_ct, g.N), dtype=np.int64)
    for i in range(g.n_out):
        ko, ii = divmod(i, g.n_ow)
        for j in range(g.n_in):
            ki, jj = divmod(j, g.n_iw)
            out[ko, ki, ii * g.n_iw + g.n_iw - 1 - jj] = Wm[i, j]
    return out


def fc_extract(polys, g):
    """polys[out_ct, N] -> y[n_out]."""
    y = np.zeros(g.n_out, dtype=np.int64)
    for i in range(g.n_out):
        ko, ii = divmod(i, g.n_ow)
        y[i] = polys[ko, ii * g.n_iw + g.n_iw - 1]
    return y


def fc_terms(B, in_ct, out_ct):
    """Output (b, o) = sum_j ct[b, j] (x) pt[o, j]."""
    row, cti, pti = [0], [], []
    for b in range(B):
        for o in range(out_ct):
            for j in range(in_ct):
                cti.append(b * in_ct + j)
                pti.append(o * in_ct + j)
            row.append(len(cti))
    return np.array(row, np.int32), np.array(cti, np.int32), np.array(pti, np.int32)


def input_degree_full_padding(H, h):
    """Highest degree of pi_x(x) for an H x H input with O = H + h - 1 (Section 3.3,
    complexity analysis): (H-1)*O + (H-1)."""
    O = H + h - 1
    return (H - 1) * O + (H - 1)


def cheetah_degree_full_padding(H, h):
    """N_1 of the complexity analysis in Section 3.3 (padded-input encoding)."""
    f = (h - 1) // 2
    return (f + H - 1) * (H + h - 1) + H + f


def corr_degree_full_padding(H, h):
    """N_2 of the complexity analysis in Section 3.3."""
    return (H + h - 1) * (H - 1)


def ceil_div(a, b):
    return -(-a // b)


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("math", "np")]


# ------------------------------------------------------------ spatial windows
# Section 3.3 splits an input whose single channel does not fit one ring element
# into windows H_w x W_w; its objective is garbled.  Reading: disjoint tiles of
# the unpadded input, tile (r, s) covering rows r*H_w.. and columns s*W_w.., each
# packed with pitch O_w = max(W_w, H_w) + h - 1 and multiplied by the same kernel
# polynomials; the product of a tile holds that tile's full correlation
# F_t[u, v] (u < H_w + h - 1, v < W_w + h - 1) at u*O_w + v, which the client
# adds into F at offset (r*H_w, s*W_w) (overlap-add: F is linear in x) and then
# crops by P.  The window is the one minimising the CPMul count
# ceil(H/H_w) * ceil(W/W_w) * cb * M subject to span_w + 1 <= N; ties go to fewer
# input ciphertexts, then larger H_w, then larger W_w.  The whole map is one of
# the admissible windows (H_w = H, W_w = W: the plain geometry), so a map that
# fits is still tiled when tiles pack more channels per polynomial and the
# count drops (64 x 64 maps with 3 channels at N = 8192: two 32 x 64 tiles with
# all channels in one polynomial, 6 CPMul for 3 outputs, against 9 unsplit).


class WindowGeometry:
    """Tiles of a conv whose input map is split into windows."""

    def __init__(self, C, M, H, W, h, P, N):
        self.C, self.M, self.H, self.W, self.h, self.P, self.N = C, M, H, W, h, P, N
        self.Hout = H + 2 * P - h + 1
        self.Wout = W + 2 * P - h + 1
        best = None
        for hw in range(1, H + 1):
            for ww in range(1, W + 1):
                O = max(ww, hw) + h - 1
                S = (hw + h - 2) * O + (ww + h - 2) + 1
                if S > N:
                    continue
                cb = -(-C // (N // S))
                tiles = -(-H // hw) * -(-W // ww)
                key = (tiles * cb * M, tiles * cb, -hw, -ww)
                if best is None or key < best[0]:
                    best = (key, hw, ww)
        if best is None:
            raise ValueError("no window fits one polynomial")
        self.Hw, self.Ww = best[1], best[2]
        self.O = max(self.Ww, self.Hw) + h - 1
        self.span = (self.Hw + h - 2) * self.O + (self.Ww + h - 2)
        self.S = self.span + 1
        self.Cw = N // self.S
        self.cb = -(-C // self.Cw)
        self.th = -(-H // self.Hw)
        self.tw = -(-W // self.Ww)
        self.tiles = self.th * self.tw

    def tile_input(self, x, t):
        """The [C, Hw, Ww] zero-extended sub-image of tile t (row-major over tiles)."""
        r, s = divmod(t, self.tw)
        sub = np.zeros((self.C, self.Hw, self.Ww), dtype=np.int64)
        blk = x[:, r * self.Hw:(r + 1) * self.Hw, s * self.Ww:(s + 1) * self.Ww]
        sub[:, :blk.shape[1], :blk.shape[2]] = blk
        return sub

    def pack_input(self, x):
        """x[C, H, W] -> [tiles, cb, N]."""
        out = np.zeros((self.tiles, self.cb, self.N), dtype=np.int64)
        for t in range(self.tiles):
            sub = self.tile_input(x, t)
            for c in range(self.C):
                k, cc = divmod(c, self.Cw)
                for i in range(self.Hw):
                    out[t, k, cc * self.S + i * self.O:cc * self.S + i * self.O + self.Ww] += sub[c, i]
        return out

    def pack_weight(self, w):
        """w[M, C, h, h] -> [M, cb, N] (pitch O, channel offsets -cc*S, negated)."""
        out = np.zeros((self.M, self.cb, self.N), dtype=np.int64)
        h = self.h
        for m in range(self.M):
            for c in range(self.C):
                k, cc = divmod(c, self.Cw)
                for a in range(h):
                    for b in range(h):
                        p = (h - 1 - a) * self.O + (h - 1 - b)
                        if cc == 0:
                            out[m, k, p] += w[m, c, a, b]
                        else:
                            out[m, k, self.N - cc * self.S + p] -= w[m, c, a, b]
        return out

    def terms(self, B):
        """Output (b, t, m) = sum_k ct[b, t, k] (x) pt[m, k]."""
        row, cti, pti = [0], [], []
        for b in range(B):
            for t in range(self.tiles):
                for m in range(self.M):
                    for k in range(self.cb):
                        cti.append((b * self.tiles + t) * self.cb + k)
                        pti.append(m * self.cb + k)
                    row.append(len(cti))
        return np.array(row, np.int32), np.array(cti, np.int32), np.array(pti, np.int32)

    def extract(self, polys):
        """Products [tiles, N] of one (b, m) -> out[Hout, Wout] by overlap-add, then crop by P."""
        h = self.h
        F = np.zeros((self.th * self.Hw + h - 1, self.tw * self.Ww + h - 1), dtype=np.int64)
        for t in range(self.tiles):
            r, s = divmod(t, self.tw)
            for u in range(self.Hw + h - 1):
                F[r * self.Hw + u, s * self.Ww:s * self.Ww + self.Ww + h - 1] += \
                    polys[t][u * self.O:u * self.O + self.Ww + h - 1]
        off = h - 1 - self.P
        return F[off:off + self.Hout, off:off + self.Wout]
