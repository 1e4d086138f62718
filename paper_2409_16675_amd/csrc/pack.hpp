// Packing of raw integer weights into one plaintext polynomial in LDS (the
// kernel polynomial pi_w of Eq. 2 per channel block, and the FC layout), for
// the kernels that pack and transform a plane in one pass.
#pragma once
#include <stdint.h>

#include "he_internal.hpp"
#include "ntt.hpp"

namespace he {

// (WPack, the layout, is declared in he_internal.hpp.)
// Scatter the weights of polynomial pp into an LDS plane that the workgroup
// has zeroed (threads tid < NT of the plane's group).
//   CONV: polynomial (m, blk) holds channels c0 = blk * Cw .. of output channel
//         m; channel c0 + cc, tap (a, b) sits at (h-1-a) O + (h-1-b), shifted
//         down by cc * S and negated for cc > 0 (X^N = -1);
//   DX:   the same with the forward weights [C][M][h][h] read transposed in
//         their channels and rotated by 180 degrees;
//   FC:   polynomial (ko, ki) holds W[ko n_ow + ii][ki n_iw + jj] at
//         ii n_iw + n_iw - 1 - jj.
template <class A, class G, class WPtr>
__device__ __forceinline__ void scatter_weights(const A &ar, typename A::V *lds, int tid, const WPack &wp, uint32_t pp,
                                                WPtr w) {
  if (wp.kind != WP_FC) {
    const uint32_t m = pp / wp.cb, blk = pp % wp.cb, hh = wp.h * wp.h;
    const uint32_t c0 = blk * wp.Cw, c1 = min(wp.C, c0 + wp.Cw);
    const uint32_t n = (c1 - c0) * hh;
    const bool dx = wp.kind == WP_CONV_DX;
    for (uint32_t id = tid; id < n; id += G::NT) {
      const uint32_t cc = id / hh, ab = id % hh, a = ab / wp.h, b = ab % wp.h;
      const size_t src = dx ? (((size_t)(c0 + cc) * wp.M + m) * wp.h + (wp.h - 1 - a)) * wp.h + (wp.h - 1 - b)
                            : ((size_t)m * wp.C + c0 + cc) * hh + ab;
      const int64_t v = w[src];
      const uint32_t pos = (wp.h - 1 - a) * wp.O + (wp.h - 1 - b);
      if (cc == 0) lds[lpad(pos)] = ar.load_signed(v);
      else lds[lpad(G::N - cc * wp.S + pos)] = ar.load_signed(-v);
    }
  } else {
    const uint32_t ko = pp / wp.in_ct, ki = pp % wp.in_ct;
    const uint32_t i0 = ko * wp.n_ow, i1 = min(wp.n_out, i0 + wp.n_ow);
    const uint32_t j0 = ki * wp.n_iw, j1 = min(wp.n_in, j0 + wp.n_iw);
    const uint32_t wi = j1 - j0, n = (i1 - i0) * wi;
    for (uint32_t id = tid; id < n; id += G::NT) {
      const uint32_t ii = id / wi, jj = id % wi;
      const int64_t v = w[(size_t)(i0 + ii) * wp.n_in + j0 + jj];
      lds[lpad(ii * wp.n_iw + wp.n_iw - 1 - jj)] = ar.load_signed(v);
    }
  }
}

}  // namespace he
