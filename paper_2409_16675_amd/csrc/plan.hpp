// Layer plan: geometry, term lists (host and device copies).
#pragma once
#include <vector>

#include "he_internal.hpp"

namespace he {

struct Plan {
  he_conv_shape shape{};
  // geometry the packing follows: the shape itself, or for an input gradient
  // (DX) the equivalent forward conv of dY (channels M -> C, map H_out x W_out,
  // padding h-1-P)
  he_conv_shape eq{};
  he_plan_info info{};
  uint32_t hk = 0;                        // polynomial-kernel side (h for CONV, Hout for DW)
  std::vector<int32_t> row, cti, pti;     // term lists (host)
  int32_t *d_terms = nullptr;             // device: row | cti | pti
  int device = 0;
  const int32_t *d_row() const { return d_terms; }
  const int32_t *d_cti() const { return d_terms + row.size(); }
  const int32_t *d_pti() const { return d_terms + row.size() + cti.size(); }
};

he_status make_plan(const Ctx &c, const he_conv_shape &s, Plan &p);

// Layout of a conv, input-gradient or FC plan's raw weights in its plaintext
// polynomials (what scatter_weights and the packing kernels follow), checked on
// the host: every packed position lies inside the N-coefficient plane and every
// weight index inside the weight tensor, else HE_EINVAL.  Weight-gradient plans
// take packed polynomials: HE_EUNSUPPORTED.
he_status weight_pack(const Plan &p, WPack &wp);

}  // namespace he

struct he_plan {
  const he::Ctx *ctx;
  he::Plan p;
};
struct he_ctx {
  he::Ctx *c;
};
