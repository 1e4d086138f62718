"""Oracle pins for spatial windows (Section 3.3: an input map that does not fit
one ring element is split into windows): the tiled packing with overlap-add
reproduces the plaintext convolution exactly through ring products at forced
small degrees, the chosen window is the cheapest feasible one (the whole map
being one of the candidates), a map that fits stays whole unless tiles lower
the count, and then the tiled layer still reproduces the convolution."""
import numpy as np
import pytest

from oracle import core, packing, plain, pyref

T = 65537


def _conv_through_windows(x, w, P, N):
    C, H, W = x.shape
    M, _, h, _ = w.shape
    g = packing.WindowGeometry(C, M, H, W, h, P, N)
    xin = g.pack_input(x)                       # [tiles, cb, N]
    pw = g.pack_weight(w)                       # [M, cb, N]
    out = np.zeros((M, g.Hout, g.Wout), dtype=np.int64)
    for m in range(M):
        prods = []
        for t in range(g.tiles):
            acc = np.zeros(N, dtype=np.int64)
            for k in range(g.cb):
                acc = (acc + core.negacyclic_mul(np.remainder(xin[t, k], T), np.remainder(pw[m, k], T), T)
                       .astype(np.int64)) % T
            prods.append(np.where(acc > T // 2, acc - T, acc))      # centred: products are small integers
        out[m] = g.extract(prods)
    return g, out


@pytest.mark.parametrize("C,M,H,W,h,P,N", [(1, 1, 12, 12, 3, 1, 64), (2, 2, 12, 10, 3, 0, 128),
                                           (3, 2, 16, 16, 5, 2, 128), (2, 1, 9, 13, 3, 1, 64)])
def test_windows_reproduce_the_convolution(C, M, H, W, h, P, N):
    g0 = np.random.Generator(np.random.PCG64(90 + H + W + N))
    x = g0.integers(-4, 5, size=(C, H, W))
    w = g0.integers(-4, 5, size=(M, C, h, h))
    g, got = _conv_through_windows(x, w, P, N)
    assert g.tiles > 1                          # these shapes need a split at this N
    assert np.array_equal(got, plain.conv2d(x, w, P))


def test_window_choice_is_the_cheapest_feasible():
    C, M, H, W, h, N = 3, 4, 64, 64, 5, 4096
    g = packing.WindowGeometry(C, M, H, W, h, 2, N)
    cost = g.tiles * g.cb * M
    for hw in range(1, H + 1):
        for ww in range(1, W + 1):
            O = max(ww, hw) + h - 1
            S = (hw + h - 2) * O + (ww + h - 2) + 1
            if S <= N:
                assert -(-H // hw) * -(-W // ww) * -(-C // (N // S)) * M >= cost
    # four 32 x 33 tiles with all three channels in one polynomial (16 CPMul)
    # beat two tiles with one channel each (24)
    assert g.span + 1 <= N and (g.tiles, g.cb) == (4, 1)


def test_no_split_when_the_whole_map_is_cheapest():
    for args in [(3, 16, 32, 32, 3, 1, 8192), (16, 32, 16, 16, 3, 1, 4096), (10, 3, 6, 6, 3, 2, 1024)]:
        C, M, H, W, h, P, N = args
        g = packing.WindowGeometry(*args)
        ref = packing.ConvGeometry(C, H, W, h, P, N)
        assert g.tiles == 1 and (g.O, g.S, g.Cw, g.cb) == (ref.O, ref.S, ref.Cw, ref.cb), args


def test_a_fitting_map_is_tiled_when_that_lowers_the_count():
    # 3 channels of 64 x 64 at N = 8192: one channel per polynomial unsplit
    # (9 CPMul), all three in each of two 32 x 64 tiles (6 CPMul)
    unsplit = packing.ConvGeometry(3, 64, 64, 5, 2, 8192)
    g = packing.WindowGeometry(3, 3, 64, 64, 5, 2, 8192)
    assert unsplit.cb * 3 == 9
    assert (g.tiles, g.cb, g.tiles * g.cb * 3) == (2, 1, 6)
    # the same at a small degree, through ring products
    C, M, H, W, h, P, N = 3, 2, 10, 10, 3, 1, 256
    assert packing.ConvGeometry(C, H, W, h, P, N).cb == 3
    g0 = np.random.Generator(np.random.PCG64(97))
    x = g0.integers(-4, 5, size=(C, H, W))
    w = g0.integers(-4, 5, size=(M, C, h, h))
    g, got = _conv_through_windows(x, w, P, N)
    assert (g.tiles, g.cb) == (2, 1)
    assert np.array_equal(got, plain.conv2d(x, w, P))
