"""Polynomial-multiplication counts of padded convolutions (Section 3.3, the
ablation on kernel and input size, Fig. 8): the planner of this library against
the blocking of Cheetah's HomConv, the prior packing the paper compares with.

Cheetah (Huang et al., USENIX Security 2022, HomConv) zero-pads the C x H x W
input to C x H' x W' (H' = H + 2P), splits it into C_w x H_w x W_w blocks with
C_w * H_w * W_w <= N, adjacent blocks overlapping by h - 1 rows and columns so
that every output lies inside one block, and multiplies each block by each of
the M packed kernels: M * ceil(C / C_w) * ceil((H' - h + 1) / (H_w - h + 1)) *
ceil((W' - h + 1) / (W_w - h + 1)) products, minimised over the block shape.

The planner here packs the unpadded input (Eq. 1-2) and splits a map that does
not fit into disjoint windows; its count is he_plan_query's n_terms.

    python -m paper_2409_16675_amd.mulcount --N 4096 8192
"""
import argparse
import json

from . import he


def _cdiv(a, b):
    return -(-a // b)


def cheetah_count(C, M, H, W, h, P, N):
    """Cheetah's HomConv product count for one image and its blocking.

    Returns (count, (C_w, H_w, W_w)); ties keep the first block shape in the
    order H_w, then W_w ascending."""
    Hp, Wp = H + 2 * P, W + 2 * P
    if Hp < h or Wp < h or h * h > N:
        raise ValueError("no block fits")
    best = None
    for hw in range(h, Hp + 1):
        for ww in range(h, Wp + 1):
            if hw * ww > N:
                break
            cw = min(C, N // (hw * ww))
            n = M * _cdiv(C, cw) * _cdiv(Hp - h + 1, hw - h + 1) * _cdiv(Wp - h + 1, ww - h + 1)
            if best is None or n < best[0]:
                best = (n, (cw, hw, ww))
    return best


def planner_count(C, M, H, W, h, P, N):
    """This library's CPMul count for one image of a forward conv, and its window."""
    i = he.he_plan_query(N, he.HE_KIND_CONV, B=1, C=C, M=M, H=H, W=W, h=h, P=P)
    return i["n_terms"], (i["Hw"], i["Ww"], i["cb"], i["tiles"])


def fig8_settings():
    """The two sweeps of the ablation: a 5 x 5 kernel on 8 x 8 ... 64 x 64 maps,
    and kernels 3 ... 11 on a 64 x 64 map; 3 input and 3 output channels, the
    padding that keeps the map size ((h - 1) / 2)."""
    a = [dict(panel="a", C=3, M=3, H=H, W=H, h=5, P=2) for H in range(8, 65, 8)]
    b = [dict(panel="b", C=3, M=3, H=64, W=64, h=h, P=(h - 1) // 2) for h in (3, 5, 7, 9, 11)]
    return a + b


def sweep(N):
    rows = []
    for s in fig8_settings():
        args = (s["C"], s["M"], s["H"], s["W"], s["h"], s["P"], N)
        ours, win = planner_count(*args)
        theirs, blk = cheetah_count(*args)
        rows.append(dict(s, N=N, planner=ours, window=win, cheetah=theirs, block=blk, ratio=theirs / ours))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, nargs="+", default=[2048, 4096, 8192])
    ap.add_argument("--json", action="store_true")
    a = ap.parse_args()
    for N in a.N:
        rows = sweep(N)
        if a.json:
            for r in rows:
                print(json.dumps(r))
            continue
        print("N = %d" % N)
        print("  panel   H   h  P | planner (Hw, Ww, cb, tiles)   | cheetah (Cw, Hw, Ww)  | ratio")
        for r in rows:
            print("  %5s %3d %3d %2d | %7d %-21s | %7d %-13s | %.2f" % (
                r["panel"], r["H"], r["h"], r["P"], r["planner"], r["window"], r["cheetah"], r["block"], r["ratio"]))


if __name__ == "__main__":
    main()
