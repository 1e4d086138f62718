"""Host-only planning and the multiplication-count study of the ablation in
Section 3.3 (Fig. 8), CPU only.

- he_plan_query (no context, no device) gives the oracle's geometry and CPMul
  counts for the sweep's settings, for windowed and input-gradient plans and
  for FC layers;
- Cheetah's HomConv blocking as counted by mulcount.cheetah_count is realised
  by brute force at small ring degrees: packing each padded block, multiplying
  it by each kernel in Z_t[X]/(X^N+1) and reading the outputs gives the
  plaintext convolution, with exactly the counted number of products;
- on the ablation's settings the two counts coincide at every ring degree,
  and on padded square maps the planner never needs more products; without
  padding, or on narrow maps, the blocking can take fewer.
"""
import numpy as np
import pytest

from oracle import core, packing, plain
from paper_2409_16675_amd import he, mulcount

T = 65537


@pytest.mark.parametrize("N", [2048, 4096, 8192])
def test_plan_query_matches_oracle_on_the_sweep(N):
    for s in mulcount.fig8_settings():
        info = he.he_plan_query(N, he.HE_KIND_CONV, B=2, C=s["C"], M=s["M"], H=s["H"], W=s["W"], h=s["h"], P=s["P"])
        g = packing.WindowGeometry(s["C"], s["M"], s["H"], s["W"], s["h"], s["P"], N)
        assert (info["Hw"], info["Ww"], info["cb"], info["tiles"], info["O"]) == (g.Hw, g.Ww, g.cb, g.tiles, g.O), s
        assert info["n_terms"] == 2 * g.tiles * g.cb * s["M"]
        assert info["n_ct_in"] == 2 * g.tiles * g.cb and info["n_ct_out"] == 2 * g.tiles * s["M"]


def test_plan_query_other_kinds_and_errors():
    # input gradient: the equivalent forward conv of dY (M -> C channels, padding h-1-P)
    info = he.he_plan_query(4096, he.HE_KIND_DX, B=1, C=3, M=4, H=64, W=64, h=5, P=2)
    g = packing.WindowGeometry(4, 3, 64, 64, 5, 2, 4096)
    assert (info["Hw"], info["Ww"], info["cb"], info["tiles"]) == (g.Hw, g.Ww, g.cb, g.tiles)
    assert info["n_terms"] == g.tiles * g.cb * 3
    fc = he.he_plan_query(8192, he.HE_KIND_FC, B=3, n_in=9216, n_out=4096)
    fg = packing.FcGeometry(9216, 4096, 8192)
    assert (fc["n_iw"], fc["n_ow"]) == (fg.n_iw, fg.n_ow)
    assert fc["n_terms"] == 3 * fg.n_cpmul
    for N in (1000, 8, 65536):
        with pytest.raises(he.HeError) as ei:
            he.he_plan_query(N, he.HE_KIND_CONV, B=1, C=1, M=1, H=4, W=4, h=3, P=1)
        assert ei.value.status == he.HE_EINVAL
    with pytest.raises(he.HeError) as ei:
        he.he_plan_query(1024, he.HE_KIND_CONV, B=1, C=1, M=1, H=4, W=4, h=3, P=3)
    assert ei.value.status == he.HE_EINVAL


def _cheetah_conv(x, w, P, N):
    """The convolution through Cheetah's HomConv blocking: returns the output and
    the number of ring products taken."""
    C, H, W = x.shape
    M, _, h, _ = w.shape
    count, (cw, hw, ww) = mulcount.cheetah_count(C, M, H, W, h, P, N)
    xp = np.zeros((C, H + 2 * P, W + 2 * P), dtype=np.int64)
    xp[:, P:P + H, P:P + W] = x
    Hout, Wout = H + 2 * P - h + 1, W + 2 * P - h + 1
    out = np.zeros((M, Hout, Wout), dtype=np.int64)
    O = hw * ww * (cw - 1) + ww * (h - 1) + h - 1
    products = 0
    for c0 in range(0, C, cw):
        for r0 in range(0, Hout, hw - h + 1):
            for s0 in range(0, Wout, ww - h + 1):
                blk = np.zeros((cw, hw, ww), dtype=np.int64)
                sub = xp[c0:c0 + cw, r0:r0 + hw, s0:s0 + ww]
                blk[:sub.shape[0], :sub.shape[1], :sub.shape[2]] = sub
                xh = np.zeros(N, dtype=np.int64)
                xh[:cw * hw * ww] = blk.reshape(-1)
                for m in range(M):
                    wh = np.zeros(N, dtype=np.int64)
                    for c in range(min(cw, C - c0)):
                        for a in range(h):
                            for b in range(h):
                                wh[O - c * hw * ww - a * ww - b] = w[m, c0 + c, a, b]
                    prod = core.negacyclic_mul(np.remainder(xh, T), np.remainder(wh, T), T).astype(np.int64)
                    products += 1
                    for i in range(min(hw - h + 1, Hout - r0)):
                        for j in range(min(ww - h + 1, Wout - s0)):
                            out[m, r0 + i, s0 + j] += prod[O + i * ww + j]
    return np.remainder(out, T), products, count


@pytest.mark.parametrize("C,M,H,W,h,P,N", [(3, 2, 6, 6, 3, 1, 64), (2, 2, 9, 7, 3, 1, 64), (3, 1, 8, 8, 5, 2, 128),
                                           (1, 2, 12, 12, 3, 0, 32)])
def test_cheetah_blocking_computes_the_convolution(C, M, H, W, h, P, N):
    g = np.random.Generator(np.random.PCG64(300 + H))
    x = g.integers(-128, 128, size=(C, H, W))
    w = g.integers(-128, 128, size=(M, C, h, h))
    got, products, count = _cheetah_conv(x, w, P, N)
    assert products == count
    assert np.array_equal(got, plain.mod_t(plain.conv2d(x, w, P), T))


@pytest.mark.parametrize("N", [256, 1024, 2048, 4096, 8192, 16384, 32768])
def test_planner_matches_cheetah_on_the_ablation_settings(N):
    # padded to keep the map size, square maps, 3 -> 3 channels: equal counts
    # (for square windows both schemes fill (H_w + h - 1)^2 coefficients per channel)
    for s in mulcount.fig8_settings():
        args = (s["C"], s["M"], s["H"], s["W"], s["h"], s["P"], N)
        assert mulcount.planner_count(*args)[0] == mulcount.cheetah_count(*args)[0], (s, N)


@pytest.mark.parametrize("N", [1024, 2048, 4096, 8192, 16384])
def test_planner_never_needs_more_products_on_padded_square_maps(N):
    # padding (h - 1) / 2 on each side and H = W, the setting of the ablation
    shapes = [(16, 16, 32, 32, 3), (64, 32, 16, 16, 3), (3, 16, 32, 32, 3), (5, 7, 24, 24, 5), (96, 96, 14, 14, 3),
              (1, 4, 100, 100, 3), (3, 64, 56, 56, 7), (3, 8, 57, 57, 7), (3, 3, 224, 224, 11)]
    for C, M, H, W, h in shapes:
        args = (C, M, H, W, h, (h - 1) // 2, N)
        assert mulcount.planner_count(*args)[0] <= mulcount.cheetah_count(*args)[0], (args, N)


@pytest.mark.parametrize("C,M,H,W,h,P,N,ours,theirs", [
    (3, 8, 57, 31, 7, 0, 2048, 40, 24),      # no padding
    (5, 7, 20, 33, 5, 0, 4096, 14, 7),       # no padding
    (3, 8, 57, 31, 7, 3, 8192, 16, 8),       # narrow map: pitch max(W, H) + h - 1 = 63 for 37 used columns
])
def test_cheetah_blocking_is_cheaper_off_the_ablation_settings(C, M, H, W, h, P, N, ours, theirs):
    # without padding the correlation packing still holds the full correlation,
    # h - 1 border rows and columns of which the convolution discards; on a
    # non-square map the row pitch of Eq. 1-2 follows the longer side
    assert mulcount.planner_count(C, M, H, W, h, P, N)[0] == ours
    assert mulcount.cheetah_count(C, M, H, W, h, P, N)[0] == theirs


def test_sweep_rows():
    rows = mulcount.sweep(4096)
    assert [r["H"] for r in rows if r["panel"] == "a"] == list(range(8, 65, 8))
    assert [r["h"] for r in rows if r["panel"] == "b"] == [3, 5, 7, 9, 11]
    for r in rows:
        assert r["ratio"] == r["cheetah"] / r["planner"] >= 1.0
