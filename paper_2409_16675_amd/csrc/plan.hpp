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

}  // namespace he

struct he_plan {
  const he::Ctx *ctx;
  he::Plan p;
};
struct he_ctx {
  he::Ctx *c;
};
