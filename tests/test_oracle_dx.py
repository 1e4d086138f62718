"""Oracle pins for the input gradient of a conv layer (Section 2: the backward
pass computes dL/dx_i = conv(w_i, dL/dx_{i+1}) with padding): the plaintext
definition against torch's own input-gradient routine and the adjoint
identity, and the packed form (the forward packing of dY with the kernel
transposed and rotated, padding h-1-P) through the oracle's ring products."""
import numpy as np
import pytest
import torch

from oracle import core, packing, plain

T = 65537


@pytest.mark.parametrize("C,M,H,h,P", [(3, 2, 6, 3, 1), (2, 4, 5, 3, 0), (1, 1, 7, 5, 2)])
def test_input_grad_matches_torch_and_adjoint(C, M, H, h, P):
    g = np.random.Generator(np.random.PCG64(70 + C + H))
    Ho = H + 2 * P - h + 1
    x = g.integers(-9, 10, size=(C, H, H))
    w = g.integers(-9, 10, size=(M, C, h, h))
    dy = g.integers(-9, 10, size=(M, Ho, Ho))
    dx = plain.conv2d_input_grad(dy, w, P, H, H)
    ref = torch.nn.grad.conv2d_input((1, C, H, H), torch.from_numpy(w).double(),
                                     torch.from_numpy(dy[None]).double(), padding=P)[0]
    assert np.array_equal(dx, ref.round().long().numpy())
    # adjoint: <conv(x, w), dy> = <x, dX(dy, w)>
    assert int((plain.conv2d(x, w, P) * dy).sum()) == int((x * dx).sum())


def test_packed_input_grad_through_ring_products():
    N, q = 1024, [core.find_primes(1024, 50, 1)[0]]
    C, M, H, h, P = 3, 2, 6, 3, 1
    Ho = H + 2 * P - h + 1
    g = np.random.Generator(np.random.PCG64(74))
    w = g.integers(-128, 128, size=(M, C, h, h))
    dy = g.integers(-128, 128, size=(M, Ho, Ho))
    # the equivalent forward conv: input dY (M channels, Ho x Ho), kernel w' [C][M], padding h-1-P
    w_eq = np.transpose(w, (1, 0, 2, 3))[:, :, ::-1, ::-1]
    geo = packing.ConvGeometry(M, Ho, Ho, h, h - 1 - P, N)
    xin = packing.pack_conv_input(dy, geo)                 # [cb, N]
    pw = packing.pack_conv_weight(np.ascontiguousarray(w_eq), geo)      # [C, cb, N]
    for c in range(C):
        acc = np.zeros(N, dtype=np.int64)
        for k in range(geo.cb):
            acc = (acc + core.negacyclic_mul(np.remainder(xin[k], T), np.remainder(pw[c, k], T), T).astype(np.int64)) % T
        got = packing.conv_extract(acc, geo)
        assert np.array_equal(got, plain.mod_t(plain.conv2d_input_grad(dy, w, P, H, H)[c], T)), c


@pytest.mark.parametrize("stride,P,H,h", [(2, 1, 9, 3), (3, 0, 11, 3), (2, 2, 8, 5)])
def test_strided_conv_matches_torch_and_subsamples_the_correlation(stride, P, H, h):
    # a stride only subsamples the full correlation that the packed product holds
    g = np.random.Generator(np.random.PCG64(95 + stride + H))
    x = g.integers(-9, 10, size=(2, H, H))
    w = g.integers(-9, 10, size=(3, 2, h, h))
    y = plain.conv2d_strided(x, w, P, stride)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x[None]).double(), torch.from_numpy(w).double(),
                                     stride=stride, padding=P)[0]
    assert np.array_equal(y, ref.round().long().numpy())
    full = plain.conv2d(x, w, P)
    assert np.array_equal(y, full[:, ::stride, ::stride])
