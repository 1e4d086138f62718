// Every ring kernel of degree 2^13 (both arithmetics, every compiled number of
// coefficients per thread).
#include "ring_kernels.hpp"

namespace he {

hipError_t run_ring_13(const Ctx &c, bool f64, int loge, Op op, const LaunchArgs &la, hipStream_t st) {
  return f64 ? run_loge<ArF64, 13>(c, loge, op, la, st) : run_loge<ArU64, 13>(c, loge, op, la, st);
}

}  // namespace he
