// The per-layer path without a caller workspace: he_corr_conv2d_noalloc runs
// the same kernels as he_corr_conv2d, with the transformed inputs and
// plaintexts in a fixed device array of this library instead of a workspace
// argument, and allocates nothing.
//
// The array lives in every GPU's copy of the code object (each device holds
// its own, at its own address, until the process ends).  Host code never uses
// its name as a device address: the address is taken once per device with
// hipGetSymbolAddress, with that device current, and kept here.
#include <mutex>

#include "plan.hpp"

namespace he {
he_status run_layer(const Ctx &c, const Plan &p, const uint64_t *ct_in, const void *plain, uint64_t *ct_out,
                    uint32_t flags, void *ws, size_t ws_bytes, hipStream_t st, const uint64_t *seed = nullptr);
size_t layer_ws_bytes(const Ctx &c, const Plan &p, uint32_t flags);
}  // namespace he

namespace {

constexpr size_t kScratchBytes = (size_t)HE_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (taken on the first call per device).
he_status scratch_ptr(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return he::fail(HE_EINVAL, "device ordinal");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return he::hip_fail(e, "hipGetDevice");
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return he::hip_fail(e, "hipSetDevice");
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    hipError_t e2 = cur != device ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return he::hip_fail(e, "scratch symbol address");
    if (e2 != hipSuccess) return he::hip_fail(e2, "hipSetDevice");
    if (!p) return he::fail(HE_EDEVICE, "scratch symbol address is null");
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return HE_OK;
}

struct Untimed {
  Untimed() { he::g_untimed = true; }
  ~Untimed() { he::g_untimed = false; }
};

}  // namespace

extern "C" he_status he_corr_conv2d_noalloc(he_ctx *ctx, const he_plan *plan, const uint64_t *ct_in,
                                            const void *plain, uint64_t *ct_out, uint32_t flags, void *stream) {
  if (!ctx || !plan || !ct_in || !plain || !ct_out) return he::fail(HE_EINVAL, "null argument");
  if (plan->ctx != ctx->c) return he::fail(HE_EINVAL, "plan belongs to another context");
  if (flags & HE_VALIDATE)
    return he::fail(HE_EINVAL, "HE_VALIDATE synchronises the stream: validate through he_corr_conv2d");
  const he::Ctx &c = *ctx->c;
  const size_t need = he::layer_ws_bytes(c, plan->p, flags);
  if (need > kScratchBytes)
    return he::fail(HE_ENOMEM, "layer needs " + std::to_string(need) + " bytes of scratch, above the fixed " +
                                   std::to_string(kScratchBytes) + " of he_corr_conv2d_noalloc");
  void *ws = nullptr;
  he_status s = scratch_ptr(c.device, &ws);
  if (s != HE_OK) return s;
  Untimed quiet;
  return he::run_layer(c, plan->p, ct_in, plain, ct_out, flags, ws, need, (hipStream_t)stream);
}
