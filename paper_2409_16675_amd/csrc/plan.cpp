// Layer planner: packing geometry and CPMul term lists for conv, weight-gradient
// and FC layers (correlation-aware packing of Section 3.3, Eq. 1 and Eq. 2).
#include "plan.hpp"

#include <algorithm>

namespace he {

static uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

static he_status make_plan_geom(const Ctx &c, const he_conv_shape &s, Plan &p);

// An input gradient (Section 2: dX = conv(w, dY) with padding) is planned as the
// forward conv of dY [B][M][H_out][W_out] with the kernel transposed in its
// channels and rotated by 180 degrees, padding h-1-P: its output map is H x W.
he_status make_plan(const Ctx &c, const he_conv_shape &s, Plan &p) {
  if (s.stride > 1 && s.kind != HE_KIND_CONV)
    return fail(HE_EUNSUPPORTED, "a stride applies to forward convolutions only");
  if (s.kind != HE_KIND_DX) {
    p.eq = s;
    return make_plan_geom(c, s, p);
  }
  if (!s.C || !s.M || !s.H || !s.W || !s.h || !s.B) return fail(HE_EINVAL, "conv sizes must be positive");
  if (s.P >= s.h) return fail(HE_EINVAL, "padding must be smaller than the kernel");
  if (s.H + 2 * s.P < s.h || s.W + 2 * s.P < s.h) return fail(HE_EINVAL, "kernel larger than padded input");
  he_conv_shape e = s;
  e.kind = HE_KIND_CONV;
  e.C = s.M;
  e.M = s.C;
  e.H = s.H + 2 * s.P - s.h + 1;
  e.W = s.W + 2 * s.P - s.h + 1;
  e.P = s.h - 1 - s.P;
  he_status st = make_plan_geom(c, e, p);
  if (st != HE_OK) return st;
  p.shape = s;
  p.eq = e;
  p.info.kind = HE_KIND_DX;
  return HE_OK;
}

he_status weight_pack(const Plan &p, WPack &wp) {
  const he_plan_info &in = p.info;
  const uint64_t N = in.N;
  wp = WPack{};
  if (in.kind == HE_KIND_CONV || in.kind == HE_KIND_DX) {
    wp.kind = in.kind == HE_KIND_DX ? WP_CONV_DX : WP_CONV;
    wp.M = p.eq.M;
    wp.C = p.eq.C;
    wp.h = p.eq.h;
    wp.O = in.O;
    wp.S = in.S;
    wp.Cw = in.Cw;
    wp.cb = in.cb;
    if (!wp.M || !wp.C || !wp.h || !wp.Cw || !wp.cb) return fail(HE_EINVAL, "weight layout: empty conv block");
    if ((uint64_t)wp.cb * wp.Cw < wp.C) return fail(HE_EINVAL, "weight layout: channel blocks miss channels");
    if (in.n_pt != wp.M * wp.cb) return fail(HE_EINVAL, "weight layout: plaintext count is not M x blocks");
    // tap (a, b) of the block's first channel sits at (h-1-a) O + (h-1-b); channel
    // cc > 0 of the block at N - cc S + that (negated): all inside [0, N) when the
    // largest tap position lies below S and N, and (channels - 1) S <= N
    const uint64_t top = (uint64_t)(wp.h - 1) * wp.O + (wp.h - 1);
    const uint64_t chans = wp.Cw < wp.C ? wp.Cw : wp.C;
    if (top >= N) return fail(HE_EINVAL, "weight layout: kernel taps beyond the ring degree");
    if (chans > 1 && (top >= wp.S || (chans - 1) * wp.S > N))
      return fail(HE_EINVAL, "weight layout: channel slots overlap or leave the plane");
  } else if (in.kind == HE_KIND_FC) {
    wp.kind = WP_FC;
    wp.n_out = p.shape.n_out;
    wp.n_in = p.shape.n_in;
    wp.n_iw = in.n_iw;
    wp.n_ow = in.n_ow;
    if (!wp.n_out || !wp.n_in || !wp.n_iw || !wp.n_ow) return fail(HE_EINVAL, "weight layout: empty FC chunk");
    wp.in_ct = (wp.n_in + wp.n_iw - 1) / wp.n_iw;
    // W[ko n_ow + ii][ki n_iw + jj] sits at ii n_iw + n_iw - 1 - jj < n_ow n_iw
    if ((uint64_t)wp.n_ow * wp.n_iw > N) return fail(HE_EINVAL, "weight layout: FC chunk beyond the ring degree");
    if (in.n_pt != ((wp.n_out + wp.n_ow - 1) / wp.n_ow) * wp.in_ct)
      return fail(HE_EINVAL, "weight layout: plaintext count is not output x input chunks");
  } else {
    return fail(HE_EUNSUPPORTED, "weight-gradient plaintexts are passed as packed polynomials (HE_PLAIN_POLY)");
  }
  return HE_OK;
}

static he_status make_plan_geom(const Ctx &c, const he_conv_shape &s, Plan &p) {
  p.shape = s;
  he_plan_info &in = p.info;
  in = he_plan_info{};
  in.kind = s.kind;
  in.N = c.N;
  const uint32_t N = c.N;
  p.row.clear();
  p.cti.clear();
  p.pti.clear();
  if (s.B == 0) return fail(HE_EINVAL, "batch must be positive");
  if (s.kind == HE_KIND_CONV || s.kind == HE_KIND_DW) {
    if (!s.C || !s.M || !s.H || !s.W || !s.h) return fail(HE_EINVAL, "conv sizes must be positive");
    if (s.H + 2 * s.P < s.h || s.W + 2 * s.P < s.h) return fail(HE_EINVAL, "kernel larger than padded input");
    if (s.P >= s.h) return fail(HE_EINVAL, "padding must be smaller than the kernel");
    const uint32_t stride = s.stride > 1 ? s.stride : 1;
    in.Hout = (s.H + 2 * s.P - s.h) / stride + 1;
    in.Wout = (s.W + 2 * s.P - s.h) / stride + 1;
    // the polynomial "kernel" is w (h x h) for CONV and dY (Hout x Hout) for DW
    uint32_t hk = s.h;
    if (s.kind == HE_KIND_DW) {
      if (in.Hout != in.Wout) return fail(HE_EUNSUPPORTED, "weight gradient needs a square output map");
      hk = in.Hout;
    }
    p.hk = hk;
    in.Hw = s.H;
    in.Ww = s.W;
    in.O = std::max(s.W, s.H) + hk - 1;
    in.span = (s.H + hk - 2) * in.O + (s.W + hk - 2);
    if (s.kind == HE_KIND_DW && in.span + 1 > N)
      return fail(HE_EUNSUPPORTED, "weight-gradient channel does not fit one polynomial");
    if (s.kind == HE_KIND_CONV) {
      // spatial windows (Section 3.3, garbled objective; reading): disjoint
      // tiles, the cheapest in CPMul count that fit, ties to fewer input
      // ciphertexts, then larger H_w, then larger W_w.  The whole map is one
      // candidate, so a map that fits is tiled only when tiles pack more
      // channels per polynomial and lower the count.
      uint64_t best[4] = {~0ull, ~0ull, ~0ull, ~0ull};
      for (uint32_t hw = 1; hw <= s.H; ++hw)
        for (uint32_t ww = 1; ww <= s.W; ++ww) {
          const uint64_t O = std::max(ww, hw) + hk - 1;
          const uint64_t S = (hw + hk - 2) * O + (ww + hk - 2) + 1;
          if (S > N) continue;
          const uint64_t cb = cdiv(s.C, (uint32_t)(N / S)), tiles = (uint64_t)cdiv(s.H, hw) * cdiv(s.W, ww);
          const uint64_t key[4] = {tiles * cb * s.M, tiles * cb, (uint64_t)(s.H - hw), (uint64_t)(s.W - ww)};
          if (std::lexicographical_compare(key, key + 4, best, best + 4)) {
            std::copy(key, key + 4, best);
            in.Hw = hw;
            in.Ww = ww;
          }
        }
      if (best[0] == ~0ull) return fail(HE_EUNSUPPORTED, "no input window fits one polynomial");
      in.O = std::max(in.Ww, in.Hw) + hk - 1;
      in.span = (in.Hw + hk - 2) * in.O + (in.Ww + hk - 2);
    }
    in.S = in.span + 1;
    in.Cw = N / in.S;
    in.cb = cdiv(s.C, in.Cw);
    in.tiles = cdiv(s.H, in.Hw) * cdiv(s.W, in.Ww);
    if (s.kind == HE_KIND_CONV) {
      const uint32_t T = in.tiles;
      in.n_ct_in = s.B * T * in.cb;
      in.n_pt = s.M * in.cb;
      in.n_ct_out = s.B * T * s.M;
      p.row.push_back(0);
      for (uint32_t b = 0; b < s.B; ++b)
        for (uint32_t t = 0; t < T; ++t)
          for (uint32_t m = 0; m < s.M; ++m) {
            for (uint32_t k = 0; k < in.cb; ++k) {
              p.cti.push_back((int32_t)((b * T + t) * in.cb + k));
              p.pti.push_back((int32_t)(m * in.cb + k));
            }
            p.row.push_back((int32_t)p.cti.size());
          }
    } else {
      // ct [B][cb + M] = ([X_b,k] blocks, [dY_b,m]); pt [B][M + cb] = ((dY-r)_b,m, (X-r)_b,k); out [M][cb]
      const uint32_t cb = in.cb, M = s.M;
      in.n_ct_in = s.B * (cb + M);
      in.n_pt = s.B * (M + cb);
      in.n_ct_out = M * cb;
      p.row.push_back(0);
      for (uint32_t m = 0; m < M; ++m)
        for (uint32_t k = 0; k < cb; ++k) {
          for (uint32_t b = 0; b < s.B; ++b) {
            p.cti.push_back((int32_t)(b * (cb + M) + k));
            p.pti.push_back((int32_t)(b * (M + cb) + m));
            p.cti.push_back((int32_t)(b * (cb + M) + cb + m));
            p.pti.push_back((int32_t)(b * (M + cb) + M + k));
          }
          p.row.push_back((int32_t)p.cti.size());
        }
    }
  } else if (s.kind == HE_KIND_FC) {
    if (!s.n_in || !s.n_out) return fail(HE_EINVAL, "FC sizes must be positive");
    uint64_t best_key[3] = {~0ull, ~0ull, ~0ull};
    for (uint32_t iw = 1; iw <= std::min(s.n_in, N); ++iw) {
      const uint32_t cap = (N + 1) / iw;
      if (cap < 2) break;
      const uint32_t ow = std::min(s.n_out, cap - 1);
      const uint32_t ict = cdiv(s.n_in, iw), oct = cdiv(s.n_out, ow);
      const uint64_t key[3] = {(uint64_t)ict * oct, ict, oct};
      if (std::lexicographical_compare(key, key + 3, best_key, best_key + 3)) {
        std::copy(key, key + 3, best_key);
        in.n_iw = iw;
        in.n_ow = ow;
      }
    }
    const uint32_t ict = cdiv(s.n_in, in.n_iw), oct = cdiv(s.n_out, in.n_ow);
    in.n_ct_in = s.B * ict;
    in.n_pt = oct * ict;
    in.n_ct_out = s.B * oct;
    p.row.push_back(0);
    for (uint32_t b = 0; b < s.B; ++b)
      for (uint32_t o = 0; o < oct; ++o) {
        for (uint32_t j = 0; j < ict; ++j) {
          p.cti.push_back((int32_t)(b * ict + j));
          p.pti.push_back((int32_t)(o * ict + j));
        }
        p.row.push_back((int32_t)p.cti.size());
      }
  } else {
    return fail(HE_EINVAL, "unknown layer kind");
  }
  in.n_terms = (uint32_t)p.cti.size();
  return HE_OK;
}

}  // namespace he
